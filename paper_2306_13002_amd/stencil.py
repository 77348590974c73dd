"""Python binding of libstencil.so (the C ABI in include/stencil.h).

Argument marshalling only: descriptors are packed into the C struct, torch
tensors are checked (device, dtype, layout, size) and passed as raw device
pointers, and every sweep runs in the library's HIP kernels.  There is no
fallback: if libstencil.so is missing or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstencil.so")

OK, E_INVAL, E_UNSUPPORTED, E_NOMEM, E_DEVICE, E_STATE = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {OK: "OK", E_INVAL: "E_INVAL", E_UNSUPPORTED: "E_UNSUPPORTED", E_NOMEM: "E_NOMEM",
                E_DEVICE: "E_DEVICE", E_STATE: "E_STATE"}
KINDS = {"heat2d5": 1, "heat3d7": 2, "poisson19": 3, "wave25": 4, "generic": 5}
DTYPES = {"f32": 1, "f64": 2}
VARIANTS = {"plain": 0, "saturated": 1, "auto": 2, "cse_sat": 3, "cse_bulk": 4, "accsat_point": 5,
            "saturated_t2": 6, "saturated_t3": 7}
VARIANT_NAMES = {v: k for k, v in VARIANTS.items()}
TUNES = {"fixed": 0, "exhaustive": 1, "model": 2}
BCS = {"dirichlet": 0, "periodic": 1}
TILE_MAPS = {"auto": 0, "natural": 1, "xcd": 2}
TILE_MAP_NAMES = {1: "natural", 2: "xcd"}
RADIUS = {"heat2d5": 1, "heat3d7": 1, "poisson19": 1, "wave25": 4}
DEFAULT_DTYPE = {"heat2d5": "f64", "heat3d7": "f64", "poisson19": "f32", "wave25": "f64", "generic": "f64"}


class StencilDesc(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("kind", ctypes.c_int32), ("dtype", ctypes.c_int32),
        ("variant", ctypes.c_int32), ("tune", ctypes.c_int32), ("bc", ctypes.c_int32),
        ("ndim", ctypes.c_int32), ("radius", ctypes.c_int32), ("n", ctypes.c_int64 * 3),
        ("pitch_y", ctypes.c_int64), ("pitch_z", ctypes.c_int64),
        ("coef", ctypes.POINTER(ctypes.c_double)), ("n_coef", ctypes.c_int32),
        ("n_taps", ctypes.c_int32), ("tap_off", ctypes.POINTER(ctypes.c_int32)),
        ("tap_cid", ctypes.POINTER(ctypes.c_int32)), ("omega", ctypes.c_double),
        ("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32), ("zblock", ctypes.c_int32),
        ("tile_map", ctypes.c_int32),
    ]


class StencilError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libstencil.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                               "python -m paper_2306_13002_amd.build")
        # torch ships its own HIP runtime under the same soname as the one
        # libstencil.so links; importing torch first makes the process load a
        # single runtime that both use (loading libstencil.so first leaves
        # torch's later initialization with a second, unusable one).
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)
        L.stencil_plan.argtypes = [ctypes.POINTER(StencilDesc), ctypes.POINTER(vp)]
        L.stencil_run.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), i32, vp]
        L.stencil_run_noalloc.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), i32, vp, vp]
        L.stencil_residual.argtypes = [vp, dp, vp]
        L.stencil_plan_config.argtypes = [vp] + [ctypes.POINTER(i32)] * 5
        L.stencil_plan_graph.argtypes = [vp, ctypes.POINTER(i32)]
        L.stencil_batch_problem_config.argtypes = [vp, i32] + [ctypes.POINTER(i32)] * 5
        L.stencil_plan_use_graphs.argtypes = [vp, i32]
        L.stencil_profile_enable.argtypes = [vp, i32]
        L.stencil_profile_read.argtypes = [vp, dp, ctypes.POINTER(i32)]
        L.stencil_destroy.argtypes = [vp]
        L.stencil_plan_batch.argtypes = [ctypes.POINTER(StencilDesc), i32, ctypes.POINTER(vp)]
        L.stencil_residuals.argtypes = [vp, dp, i32, vp]
        fp = ctypes.POINTER(ctypes.c_float)
        L.stencil_candidates.argtypes = [ctypes.POINTER(StencilDesc), i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.stencil_features.argtypes = [ctypes.POINTER(StencilDesc), i32, i32, i32, i32, i32, fp]
        L.stencil_mlp_train.argtypes = [fp, fp, i32, fp, i32, ctypes.c_float, fp, fp, vp]
        L.stencil_mlp_predict.argtypes = [fp, fp, i32, fp, vp]
        L.stencil_prepare.argtypes = [ctypes.POINTER(StencilDesc)]
        L.stencil_prepare.restype = ctypes.c_int
        L.stencil_stream.argtypes = [i32, vp, vp, vp, vp, ctypes.c_int64, i32, i32, i32, vp]
        L.stencil_stream.restype = ctypes.c_int
        for f in (L.stencil_plan, L.stencil_run, L.stencil_run_noalloc, L.stencil_residual, L.stencil_plan_config,
                  L.stencil_plan_graph,
                  L.stencil_plan_use_graphs, L.stencil_batch_problem_config,
                  L.stencil_profile_enable, L.stencil_profile_read, L.stencil_destroy, L.stencil_plan_batch,
                  L.stencil_residuals, L.stencil_candidates, L.stencil_features, L.stencil_mlp_train,
                  L.stencil_mlp_predict):
            f.restype = ctypes.c_int
        L.stencil_last_error.restype = ctypes.c_char_p
        L.stencil_last_error.argtypes = []
        L.stencil_version.restype = ctypes.c_char_p
        L.stencil_version.argtypes = []
        _lib = L
    return _lib


def last_error() -> str:
    return lib().stencil_last_error().decode()


def _check(st: int):
    if st != OK:
        raise StencilError(st, last_error())


def make_desc(kind: str, n: Sequence[int], dtype: Optional[str] = None, variant: str = "auto",
              tune: str = "fixed", bc: str = "dirichlet", coef: Optional[Sequence[float]] = None,
              taps: Optional[Sequence[Sequence[int]]] = None, cids: Optional[Sequence[int]] = None,
              radius: Optional[int] = None, omega: float = 0.8, tile: Sequence[int] = (0, 0, 0),
              pitch: Sequence[int] = (0, 0), tile_map: str = "auto"):
    """Pack a stencil_desc.  Returns (desc, keepalive) -- keep the second
    object alive until stencil_plan has copied the host arrays."""
    d = StencilDesc()
    d.struct_size = ctypes.sizeof(StencilDesc)
    d.kind = KINDS[kind]
    d.dtype = DTYPES[dtype or DEFAULT_DTYPE[kind]]
    d.variant = VARIANTS[variant]
    d.tune = TUNES[tune]
    d.bc = BCS[bc]
    d.ndim = 2 if kind == "heat2d5" else 3
    d.radius = int(radius if radius is not None else RADIUS.get(kind, 1))
    nn = list(n) + [1] * (3 - len(n))
    for a in range(3):
        d.n[a] = int(nn[a])
    d.pitch_y, d.pitch_z = int(pitch[0]), int(pitch[1])
    keep = []
    if coef is not None:
        ca = (ctypes.c_double * len(coef))(*[float(c) for c in coef])
        keep.append(ca)
        d.coef = ctypes.cast(ca, ctypes.POINTER(ctypes.c_double))
        d.n_coef = len(coef)
    if taps is not None:
        flat = [int(v) for t in taps for v in t]
        ta = (ctypes.c_int32 * len(flat))(*flat)
        ci = (ctypes.c_int32 * len(cids))(*[int(c) for c in cids])
        keep += [ta, ci]
        d.tap_off = ctypes.cast(ta, ctypes.POINTER(ctypes.c_int32))
        d.tap_cid = ctypes.cast(ci, ctypes.POINTER(ctypes.c_int32))
        d.n_taps = len(taps)
    d.omega = float(omega)
    d.tile_x, d.tile_y, d.zblock = (int(v) for v in tile)
    d.tile_map = TILE_MAPS[tile_map]
    return d, keep


def plan_status(desc: StencilDesc) -> tuple[int, Optional[int]]:
    """Call stencil_plan; returns (status, handle or None) without raising."""
    h = ctypes.c_void_p()
    st = lib().stencil_plan(ctypes.byref(desc), ctypes.byref(h))
    return st, (h.value if st == OK else None)


def _stream_handle(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


class _GridLayout:
    """The padded layout of one descriptor's grids and the checks of the
    tensors handed to the library for it."""

    def __init__(self, kind: str, n: Sequence[int], **kw):
        self.kind = kind
        self.n = tuple(int(v) for v in n)
        self.dtype = kw.get("dtype") or DEFAULT_DTYPE[kind]
        self.radius = int(kw.get("radius") if kw.get("radius") is not None else RADIUS.get(kind, 1))
        self.pitch = tuple(kw.get("pitch", (0, 0)))
        # fixed per layout; the tensor checks of every run compare against them
        self._span_n = self._span()
        self._shape_n = self.padded_shape()

    def padded_shape(self):
        r = self.radius
        if self.kind == "heat2d5":
            return (self.n[1] + 2 * r, self.n[0] + 2 * r)
        return (self.n[2] + 2 * r, self.n[1] + 2 * r, self.n[0] + 2 * r)

    def _span(self):
        r = self.radius
        PX, PY = self.n[0] + 2 * r, self.n[1] + 2 * r
        py = self.pitch[0] or PX
        if self.kind == "heat2d5":
            return (PY - 1) * py + PX
        PZ = self.n[2] + 2 * r
        pz = self.pitch[1] or py * PY
        return (PZ - 1) * pz + (PY - 1) * py + PX

    def _check_tensor(self, t, dtype_name: str, what: str):
        import torch
        want = torch.float32 if dtype_name == "f32" else torch.float64
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{what} must be a torch tensor")
        if not t.is_cuda:
            raise ValueError(f"{what} must be a device (cuda) tensor")
        if t.dtype != want:
            raise TypeError(f"{what} must be {want}, got {t.dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{what} must be contiguous (use pitch= for padded rows)")
        if t.numel() < self._span_n:
            raise ValueError(f"{what} holds {t.numel()} elements, the padded grid spans {self._span_n}")
        if self.pitch == (0, 0) and t.shape != self._shape_n and t.dim() != 1:
            raise ValueError(f"{what} shape {tuple(t.shape)} != padded shape {self._shape_n}")
        return ctypes.c_void_p(t.data_ptr())

    def _pointers(self, fields, coef_arrays):
        """(field pointer array, coefficient pointer array or None)."""
        if len(fields) != 2:
            raise ValueError("two field tensors are required")
        fp = (ctypes.c_void_p * 2)(*[self._check_tensor(f, self.dtype, f"fields[{i}]") for i, f in enumerate(fields)])
        cp = None
        if self.kind == "poisson19":
            if coef_arrays is None or len(coef_arrays) != 12:
                raise ValueError("poisson19 needs 12 coefficient tensors")
            cp = (ctypes.c_void_p * 12)(*[self._check_tensor(c, "f32", f"coef[{i}]") for i, c in enumerate(coef_arrays)])
        elif self.kind == "wave25":
            if coef_arrays is None or len(coef_arrays) != 1:
                raise ValueError("wave25 needs coef_arrays = [vsq]")
            cp = (ctypes.c_void_p * 1)(self._check_tensor(coef_arrays[0], "f64", "vsq"))
        return fp, cp


class Plan(_GridLayout):
    """A built plan.  Grids are padded torch tensors (see include/stencil.h)."""

    def __init__(self, kind: str, n: Sequence[int], **kw):
        super().__init__(kind, n, **kw)
        desc, keep = make_desc(kind, n, **kw)
        h = ctypes.c_void_p()
        _check(lib().stencil_plan(ctypes.byref(desc), ctypes.byref(h)))
        del keep
        self._h = h

    # calls ---------------------------------------------------------------
    def run(self, fields, coef_arrays=None, iterations: int = 1, stream=None):
        """Run `iterations` sweeps (asynchronous on `stream`, default: torch's
        current stream).  For wave25, returns (older, newer) tensors."""
        fp, cp = self._pointers(fields, coef_arrays)
        _check(lib().stencil_run(self._h, fp, cp, int(iterations), ctypes.c_void_p(_stream_handle(stream))))
        if self.kind == "wave25":
            return (fields[1], fields[0]) if iterations % 2 == 1 else (fields[0], fields[1])
        return fields[0]

    def run_noalloc(self, fields, coef_arrays=None, iterations: int = 1, residual=None, stream=None):
        """stencil_run_noalloc: the sweeps of run() with the library's device
        scratch; the FP64 residual goes to `residual` (a float64 device
        tensor, element 0), or nowhere if None.  Never synchronizes."""
        fp, cp = self._pointers(fields, coef_arrays)
        import torch

        rp = None
        if residual is not None:
            if residual.dtype != torch.float64 or not residual.is_cuda or residual.numel() < 1:
                raise ValueError("residual must be a float64 device tensor with at least one element")
            rp = ctypes.c_void_p(residual.data_ptr())
        _check(lib().stencil_run_noalloc(self._h, fp, cp, int(iterations), rp,
                                         ctypes.c_void_p(_stream_handle(stream))))
        if self.kind == "wave25":
            return (fields[1], fields[0]) if iterations % 2 == 1 else (fields[0], fields[1])
        return fields[0]

    def residual(self, stream=None) -> float:
        out = ctypes.c_double()
        _check(lib().stencil_residual(self._h, ctypes.byref(out), ctypes.c_void_p(_stream_handle(stream))))
        return out.value

    def config(self) -> dict:
        v, tx, ty, zb, m = (ctypes.c_int32() for _ in range(5))
        _check(lib().stencil_plan_config(self._h, ctypes.byref(v), ctypes.byref(tx), ctypes.byref(ty), ctypes.byref(zb),
                                         ctypes.byref(m)))
        return {"variant": VARIANT_NAMES[v.value], "tile": (tx.value, ty.value, zb.value),
                "tile_map": TILE_MAP_NAMES.get(m.value, m.value)}

    def use_graphs(self, enable: bool = True):
        """Replay repeated identical runs from captured HIP graphs."""
        _check(lib().stencil_plan_use_graphs(self._h, 1 if enable else 0))

    def graph_iterations(self) -> int:
        """Iteration count of the run replayed from captured graphs (0: none)."""
        t = ctypes.c_int32()
        _check(lib().stencil_plan_graph(self._h, ctypes.byref(t)))
        return t.value

    def profile(self, enable: bool = True):
        _check(lib().stencil_profile_enable(self._h, 1 if enable else 0))

    def profile_read(self):
        ms, n = ctypes.c_double(), ctypes.c_int32()
        _check(lib().stencil_profile_read(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().stencil_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class BatchPlan:
    """Many independent HEAT3D7 grids run as one graph (stencil_plan_batch).
    problems: list of interior extents (nx, ny, nz); every problem uses the
    same coefficients and the form/tuning options given here."""

    def __init__(self, problems, coef=(0.4, 0.1), **kw):
        self.n = [tuple(int(v) for v in p) for p in problems]
        descs = (StencilDesc * len(self.n))()
        keep = []
        for i, n in enumerate(self.n):
            d, k = make_desc("heat3d7", n, coef=coef, **kw)
            descs[i] = d
            keep.append(k)
        h = ctypes.c_void_p()
        _check(lib().stencil_plan_batch(descs, len(self.n), ctypes.byref(h)))
        del keep
        self._h = h
        self._plans = [Plan.__new__(Plan) for _ in self.n]
        for p, n in zip(self._plans, self.n):  # layout checkers only (no library handle)
            _GridLayout.__init__(p, "heat3d7", n, dtype="f64", radius=1)
            p._h = None

    def run(self, fields, iterations: int = 1, stream=None):
        """fields: one (state, scratch) pair of padded tensors per problem."""
        if len(fields) != len(self.n):
            raise ValueError(f"{len(self.n)} field pairs are required")
        flat = []
        for i, (pair, chk) in enumerate(zip(fields, self._plans)):
            flat += [chk._check_tensor(pair[0], "f64", f"problem {i} fields[0]"),
                     chk._check_tensor(pair[1], "f64", f"problem {i} fields[1]")]
        fp = (ctypes.c_void_p * len(flat))(*flat)
        _check(lib().stencil_run(self._h, fp, None, int(iterations), ctypes.c_void_p(_stream_handle(stream))))

    def config(self) -> dict:
        """Form and launch shape of the first size class, and every class's
        (form, launch shape, number of problems) under "classes"."""
        v, tx, ty, zb, m = (ctypes.c_int32() for _ in range(5))
        _check(lib().stencil_plan_config(self._h, ctypes.byref(v), ctypes.byref(tx), ctypes.byref(ty), ctypes.byref(zb),
                                         ctypes.byref(m)))
        classes = [{"variant": c["variant"], "tile": c["tile"], "problems": len(c["problems"])} for c in self.classes()]
        return {"variant": VARIANT_NAMES[v.value], "tile": (tx.value, ty.value, zb.value), "tile_map": "batch",
                "classes": classes}

    def problem_config(self, i: int) -> dict:
        """Size class, form and launch shape of problem i."""
        c, v, tx, ty, zb = (ctypes.c_int32() for _ in range(5))
        _check(lib().stencil_batch_problem_config(self._h, int(i), ctypes.byref(c), ctypes.byref(v), ctypes.byref(tx),
                                                  ctypes.byref(ty), ctypes.byref(zb)))
        return {"size_class": c.value, "variant": VARIANT_NAMES[v.value], "tile": (tx.value, ty.value, zb.value)}

    def classes(self) -> list:
        """One entry per size class: its form, launch shape and problem indices."""
        out = {}
        for i in range(len(self.n)):
            pc = self.problem_config(i)
            e = out.setdefault(pc["size_class"], {"variant": pc["variant"], "tile": pc["tile"], "problems": []})
            e["problems"].append(i)
        return [out[k] for k in sorted(out)]

    def residuals(self, stream=None):
        out = (ctypes.c_double * len(self.n))()
        _check(lib().stencil_residuals(self._h, out, len(self.n), ctypes.c_void_p(_stream_handle(stream))))
        return list(out)

    def residual(self, stream=None) -> float:
        out = ctypes.c_double()
        _check(lib().stencil_residual(self._h, ctypes.byref(out), ctypes.c_void_p(_stream_handle(stream))))
        return out.value

    def profile(self, enable: bool = True):
        _check(lib().stencil_profile_enable(self._h, 1 if enable else 0))

    def profile_read(self):
        ms, n = ctypes.c_double(), ctypes.c_int32()
        _check(lib().stencil_profile_read(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().stencil_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


# ---------------------------------------------------------------- cost model
N_FEATURES = 24
N_MLP_PARAMS = 5825


def candidates(kind: str, n, **kw):
    """The launch candidates the tuners consider: list of
    (variant, (tile_x, tile_y, zblock), tile_map) with names."""
    d, keep = make_desc(kind, n, **kw)
    cnt = ctypes.c_int32()
    _check(lib().stencil_candidates(ctypes.byref(d), 0, None, ctypes.byref(cnt)))
    buf = (ctypes.c_int32 * (5 * max(1, cnt.value)))()
    _check(lib().stencil_candidates(ctypes.byref(d), cnt.value, buf, ctypes.byref(cnt)))
    out = []
    for i in range(cnt.value):
        v, tx, ty, zb, m = buf[5 * i:5 * i + 5]
        out.append((VARIANT_NAMES[v], (tx, ty, zb), TILE_MAP_NAMES[m]))
    return out


def prepare(kind: str, n, **kw):
    """Compile the generated kernels the tuners may try (GENERIC; else no-op)."""
    d, keep = make_desc(kind, n, **kw)
    _check(lib().stencil_prepare(ctypes.byref(d)))


def features(kind: str, n, cand, **kw):
    """The 24 cost-model features of a stencil run with one candidate."""
    import numpy as np
    d, keep = make_desc(kind, n, **kw)
    v, (tx, ty, zb), m = cand
    out = (ctypes.c_float * N_FEATURES)()
    _check(lib().stencil_features(ctypes.byref(d), VARIANTS[v], tx, ty, zb, TILE_MAPS[m], out))
    return np.array(out[:], dtype=np.float32)


def _fptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def mlp_train(X, y, init, epochs: int, lr: float = 1e-3, stream=None):
    """Train the cost-model MLP on the device (see stencil_mlp_train).
    Returns (model vector of 24 + 24 + 5825 floats, loss before each step)."""
    import numpy as np
    X = np.ascontiguousarray(X, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    th = np.ascontiguousarray(init, dtype=np.float32)
    if X.ndim != 2 or X.shape[1] != N_FEATURES or y.shape != (X.shape[0],) or th.shape != (N_MLP_PARAMS,):
        raise ValueError("X must be n x 24, y n, init 5825")
    model = np.zeros(2 * N_FEATURES + N_MLP_PARAMS, dtype=np.float32)
    loss = np.zeros(max(1, epochs), dtype=np.float32)
    _check(lib().stencil_mlp_train(_fptr(X), _fptr(y), X.shape[0], _fptr(th), int(epochs), float(lr), _fptr(model),
                                   _fptr(loss), ctypes.c_void_p(_stream_handle(stream))))
    return model, loss[:epochs]


def mlp_predict(model, X, stream=None):
    import numpy as np
    model = np.ascontiguousarray(model, dtype=np.float32)
    X = np.ascontiguousarray(X, dtype=np.float32)
    out = np.zeros(X.shape[0], dtype=np.float32)
    _check(lib().stencil_mlp_predict(_fptr(model), _fptr(X), X.shape[0], _fptr(out),
                                     ctypes.c_void_p(_stream_handle(stream))))
    return out


# ---------------------------------------------------------------- streaming kernels of known traffic
STREAM_OPS = {"copy": 0, "3r1w": 1}


def stream(op: str, a, b, c, d, width: int = 1, nt_loads: bool = False, nt_stores: bool = False, grid: int = 0,
           stream=None):
    """Enqueue one streaming kernel of known traffic (see stencil_stream):
    op "copy" writes d = a, "3r1w" writes d = fma(c, a, 2a - b); a, b, c, d
    are float64 CUDA tensors of one size (b, c may be None for "copy"; d may
    be b).  Asynchronous on the current stream."""
    import torch
    n = a.numel()
    for t in (a, b, c, d):
        if t is not None and (t.dtype != torch.float64 or not t.is_cuda or t.numel() != n or not t.is_contiguous()):
            raise ValueError("stream: contiguous float64 CUDA tensors of one size are required")
    ptr = lambda t: ctypes.c_void_p(t.data_ptr() if t is not None else 0)
    flags = (1 if nt_loads else 0) | (2 if nt_stores else 0)
    _check(lib().stencil_stream(STREAM_OPS[op], ptr(a), ptr(b), ptr(c), ptr(d), n, int(width), flags, int(grid),
                                ctypes.c_void_p(_stream_handle(stream))))
