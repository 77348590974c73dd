"""Benchmark: grid-point updates/s of the stencil sweeps on one MI355X.

Default workload (the headline): the radius-4 25-point leapfrog wave update,
FP64, 512^3 interior + 4-cell halo, 10 steps per benchmark step, saturated
form at its autotuned launch shape, the plain form timed beside it.  One
step = one stencil_run of 10 steps plus the FP64 residual read-back; inputs
are resident in HBM before timing starts.  Before timing, each form runs the
workload once from the seeded inputs; the CPU-baseline leg runs the oracle on
light-cone crops of that run and reports the max relative error (saturated
<= 1e-12, plain bit-identical) beside the oracle's own throughput.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Prints one JSON line.  The headline line also carries secondary objects:
streaming ceilings of the sweeps' access shapes, poisson19 129x129x257 (F32
storage, Infinity-Cache resident), heat3d7 160^3, the 64-grid heat3d7
batch, and heat2d5 256^2 (one launch per sweep and fused sweeps, with the
oracle's one-core and all-core rates).  --workload poisson19 | heat3d7 | heat2d5 | batch | generic | stream |
copy times one of them alone (for profiling runs); --workload lhs times the
saturator's block-tridiagonal assembly program (162^3, 75 statements) in the
five forms of the paper's ablation.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X published HBM3E bandwidth
INFINITY_CACHE_BYTES = 256 << 20  # MI355X Infinity Cache (MALL)
FP64_VECTOR_PEAK_TFLOPS = 78.6  # MI355X published FP64 vector peak
# Launch shapes come from the library's exhaustive autotuner at plan time
# (outside the timed region), separately for each form.
TUNE = "exhaustive"


def sha256_of(paths):
    """sha256 of one file, or of several files' bytes concatenated in order."""
    h = hashlib.sha256()
    for path in ([paths] if isinstance(paths, str) else paths):
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def read_traffic(kernel_tag: str, source: str):
    """HBM bytes per launch from a committed rocprofv3 --pmc summary, or None
    when absent or taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", f"{kernel_tag}_pmc.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    srcs = [source] if isinstance(source, str) else list(source)
    if kv.get("kernel_source_sha256") != sha256_of([os.path.join(ROOT, "paper_2306_13002_amd", "csrc", f) for f in srcs]):
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def setup_workload(name, variant, dev, torch, synth, Plan, plan_kw=None):
    """Returns (plan, run_step, reset, points_per_step, sweeps_per_step, meta)."""
    pk = dict(tune=TUNE)
    pk.update(plan_kw or {})
    if name == "poisson19":
        p0, cf = synth.poisson19_inputs()
        n = (127, 127, 255)
        plan = Plan("poisson19", n, variant=variant, omega=0.8, **pk)
        f = [torch.tensor(p0, device=dev), torch.empty(p0.shape, dtype=torch.float32, device=dev)]
        cs = [torch.tensor(c, device=dev) for c in cf]
        base = f[0].clone()
        T = 20

        def step():
            plan.run(f, cs, iterations=T)
            return plan.residual()

        def reset():
            f[0].copy_(base)

        meta = dict(workload="poisson19 19-point variable-coefficient pressure relaxation, 129x129x257 incl. "
                             "boundary, F32 storage / FP64 arithmetic, omega 0.8, 20 sweeps + FP64 residual",
                    grid_total=[129, 129, 257], interior=list(n), iterations=T, bytes_per_update=56,
                    kernel_tag={"saturated": "poisson19_sat_129x129x257", "saturated_t2": "poisson19_sat2_129x129x257"}
                    .get(variant, "poisson19_plain_129x129x257"),
                    source="poisson19.hip", storage="f32", sweeps_per_launch=2 if variant == "saturated_t2" else 1)
        return plan, step, reset, n[0] * n[1] * n[2] * T, T, meta
    if name == "wave25":
        a, b, v = synth.wave25_inputs(512)
        n = (512, 512, 512)
        plan = Plan("wave25", n, variant=variant, coef=synth.WAVE25_COEF, **pk)
        f = [torch.tensor(a, device=dev), torch.tensor(b, device=dev)]
        vs = [torch.tensor(v, device=dev)]
        del a, b, v
        T = 10

        def step():
            plan.run(f, vs, iterations=T)
            return plan.residual()

        meta = dict(workload="wave25 radius-4 leapfrog, 512^3 interior + 4-cell halo, FP64, 10 steps + residual",
                    interior=list(n), iterations=T, bytes_per_update=32,
                    kernel_tag=f"wave25_{'sat' if variant == 'saturated' else 'plain'}_512c",
                    source=("wave25.hip", "common.hpp"), storage="f64")
        return plan, step, (lambda: None), n[0] * n[1] * n[2] * T, T, meta
    if name in ("heat2d5", "heat3d7"):
        if name == "heat2d5":
            u0 = synth.heat2d5_input(256)
            n, T, coef = (256, 256), 10, (0.6, 0.1)
        else:
            n, T, coef = (160, 160, 160), 50, (0.4, 0.1)
            u0 = synth.heat3d7_input(*n)
        plan = Plan(name, n, variant=variant if name == "heat3d7" else "plain", coef=coef, **pk)
        f = [torch.tensor(u0, device=dev), torch.empty(u0.shape, dtype=torch.float64, device=dev)]
        base = f[0].clone()

        def step():
            plan.run(f, iterations=T)
            return plan.residual()

        def reset():
            f[0].copy_(base)

        pts = 1
        for v in n:
            pts *= v
        meta = dict(workload=f"{name} Jacobi heat, interior {n}, FP64, {T} sweeps + residual", interior=list(n),
                    iterations=T, bytes_per_update=16, kernel_tag=f"{name}_{variant}", source="heat.hip",
                    storage="f64", sweeps_per_launch={"saturated_t2": 2, "saturated_t3": 3}.get(variant, 1))
        fuse = plan.config()["tile"][2] if name == "heat2d5" else 1
        if fuse > 1:  # plain sweeps fused per launch (the first launch of a run takes the remainder)
            meta.update(kernel_tag="heat2d5_fused", sweeps_per_launch=fuse)
        return plan, step, reset, pts * T, T, meta
    if name == "generic":
        w = synth.generic_box_workload()
        n, r, T = w["n"], w["radius"], 4
        plan = Plan("generic", n, variant=variant, dtype="f64", radius=r, coef=w["coef"], taps=w["taps"],
                    cids=w["cids"], **pk)
        u0 = synth.generic_input(n, r, "f64", stream=901)
        f = [torch.tensor(u0, device=dev), torch.empty(u0.shape, dtype=torch.float64, device=dev)]
        base = f[0].clone()
        del u0

        def step():
            plan.run(f, iterations=T)
            return plan.residual()

        def reset():
            f[0].copy_(base)

        n_taps = len(w["taps"])
        n_groups = len(set((t[2], c) for t, c in zip(w["taps"], w["cids"])))
        # FP64 operations per point update: plain = one multiply and one add per
        # tap (the first add absent); saturated = the taps of a group summed
        # (n_taps - n_groups adds) and one FMA per group
        if variant == "plain":
            instr, flops = 2 * n_taps - 1, 2 * n_taps - 1
        else:
            instr, flops = n_taps, (n_taps - n_groups) + 2 * n_groups
        meta = dict(workload=f"generic box stencil r={r}, {n_taps} taps, {len(w['coef'])} shared coefficients "
                             f"(symmetric), FP64, interior {n}, {T} sweeps + residual", interior=list(n),
                    iterations=T, bytes_per_update=16, kernel_tag=f"generic_box3_{variant}",
                    source=("generic.hip",) if variant == "plain" else ("rtc.cpp", "generic_body.hpp", "common.hpp"),
                    storage="f64", bound="alu", flops_per_update=flops, instr_per_update=instr)
        return plan, step, reset, n[0] * n[1] * n[2] * T, T, meta
    if name == "batch":
        from paper_2306_13002_amd.stencil import BatchPlan
        sizes = synth.heat3d7_batch_sizes()
        T = 50
        us = [synth.heat3d7_input(*n, stream=1 + b) for b, n in enumerate(sizes)]
        fs = [(torch.tensor(u, device=dev), torch.empty(u.shape, dtype=torch.float64, device=dev)) for u in us]
        pts = sum(n[0] * n[1] * n[2] for n in sizes)
        if variant in ("saturated", "saturated_t2", "saturated_t3"):  # the batched graph, classes tuned
            plan = BatchPlan(sizes, tune=TUNE, variant=variant)

            def step():
                plan.run(fs, iterations=T)
                return plan.residual()
        else:  # baseline: 64 separate plain runs at the default launch shape
            plans = [Plan("heat3d7", n, variant="plain", coef=(0.4, 0.1)) for n in sizes]

            class _Seq:
                def profile(self, on):
                    self.ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))

                def profile_read(self):
                    self.ev[1].synchronize()
                    return self.ev[0].elapsed_time(self.ev[1]), T

                def config(self):
                    return plans[0].config()

                def close(self):
                    for q in plans:
                        q.close()

            plan = _Seq()

            def step():
                plan.ev[0].record()
                for q, f in zip(plans, fs):
                    q.run(list(f), iterations=T)
                plan.ev[1].record()
                return sum(q.residual() for q in plans)

        class _BatchCfg:
            pass

        meta = dict(workload="64 independent heat3d7 FP64 grids, edges 32..160 (seeded), 50 sweeps each + "
                             "residuals; batched graph vs 64 separate plain runs",
                    interior=[len(sizes), pts], iterations=T, bytes_per_update=16, kernel_tag="heat3d7_batch",
                    source="heat.hip", storage="f64",
                    sweeps_per_launch={"saturated_t2": 2, "saturated_t3": 3}.get(variant, 1))
        return plan, step, (lambda: None), pts * T, T, meta
    if name == "copy":
        # plain device-to-device copy of 1 GiB: the streaming ceiling, and the
        # known-size kernel that calibrates the HBM byte counters
        nbytes = 1 << 30
        src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)

        class _CopyPlan:
            def profile(self, on):
                self.ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))

            def profile_read(self):
                self.ev[1].synchronize()
                return self.ev[0].elapsed_time(self.ev[1]), 1

            def config(self):
                return {"tile": (0, 0, 0)}

            def close(self):
                pass

        plan = _CopyPlan()

        def step():
            plan.ev[0].record()
            dst.copy_(src)
            plan.ev[1].record()
            return None

        meta = dict(workload="device copy, 1 GiB read + 1 GiB write (torch copy_)", interior=[nbytes // 8],
                    iterations=1, bytes_per_update=16, kernel_tag="copy_1GiB", source="support.hip", storage="f64")
        return plan, step, (lambda: None), nbytes // 8, 1, meta
    raise SystemExit(f"unknown workload {name}")


def time_variant(name, variant, steps, warmup, dev, torch, synth, Plan, plan_kw=None):
    plan, step, reset, pts, T, meta = setup_workload(name, variant, dev, torch, synth, Plan, plan_kw)
    # Each timed step continues the iteration from the previous state: the
    # same work on the same grid (the restore copy is done once, untimed).
    r = timed(plan, step, reset, steps, warmup, torch)
    cfg = plan.config()
    plan.close()
    return dict(wall=r["wall"], pts=pts, sweep_ms=r["sweep_ms"], sweeps=r["sweeps"], resid=r["resid"], meta=meta,
                cfg=cfg, T=T, sweep_ms_median=r["sweep_ms_median"], sweep_ms_best=r["sweep_ms_best"])


def cpu_threads():
    """Host threads for the all-cores oracle run: the cores this process may
    use, at most 16 (one GPU's share of a host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def all_cores(call, pts_per_call, one_s, label):
    """The same oracle call run by one thread per core at once (the oracle's
    C body runs without the GIL), each on its own copy of the inputs, for
    about 10 s; returns the aggregate rate."""
    import threading

    n = cpu_threads()
    reps = max(1, int(10.0 / max(one_s, 1e-3)))
    barrier = threading.Barrier(n + 1)

    def work():
        barrier.wait()
        for _ in range(reps):
            call()

    ts = [threading.Thread(target=work) for _ in range(n)]
    for t in ts:
        t.start()
    barrier.wait()
    t0 = time.perf_counter()
    for t in ts:
        t.join()
    dt = time.perf_counter() - t0
    return dict(value=n * reps * pts_per_call / dt, cores=n,
                sample=f"{n} threads, each {reps} x ({label}), {dt:.1f} s")


def cpu_baseline(name):
    """Time the CPU oracle (single thread, as written) on a bounded sample,
    and the same calls on every core at once ("all_cores")."""
    import numpy as np

    import oracle
    from paper_2306_13002_amd import synth

    if name == "poisson19":
        p0, cf = synth.poisson19_inputs()
        oracle.poisson19(p0, cf, 0.8, 1, mode="F32STORE")  # warm the oracle library and caches
        t = time.perf_counter()
        oracle.poisson19(p0, cf, 0.8, 8, mode="F32STORE")
        one = (time.perf_counter() - t) / 8
        k = max(2, min(4000, int(20.0 / max(one, 1e-3))))
        t = time.perf_counter()
        oracle.poisson19(p0, cf, 0.8, k, mode="F32STORE")
        dt = time.perf_counter() - t
        pts = 127 * 127 * 255 * k
        ac = all_cores(lambda: oracle.poisson19(p0, cf, 0.8, 8, mode="F32STORE"), 127 * 127 * 255 * 8, 8 * one,
                       "8 sweeps of the full grid")
        return dict(value=pts / dt, unit="grid-point updates/s", cores=1, kind="oracle",
                    sample=f"full 129x129x257 grid, {k} sweeps (F32STORE mode), {dt:.1f} s, single thread",
                    all_cores=ac)
    if name == "wave25":
        a, b, v = synth.wave25_inputs(128, 128, 128)
        t = time.perf_counter()
        oracle.wave25(a, b, v, synth.WAVE25_COEF, 2)
        one = (time.perf_counter() - t) / 2
        k = max(1, min(500, int(10.0 / max(one, 1e-3))))
        t = time.perf_counter()
        oracle.wave25(a, b, v, synth.WAVE25_COEF, k)
        dt = time.perf_counter() - t
        ac = all_cores(lambda: oracle.wave25(a, b, v, synth.WAVE25_COEF, 2), 128 ** 3 * 2, 2 * one,
                       "2 steps of the 128^3 crop")
        return dict(value=128 ** 3 * k / dt, unit="grid-point updates/s", cores=1, kind="oracle",
                    sample=f"128^3 crop of the same recipe, {k} steps, {dt:.1f} s, single thread", all_cores=ac)
    if name == "generic":
        w = synth.generic_box_workload()
        n = (64, 64, 64)
        u0 = synth.generic_input(n, w["radius"], "f64", stream=901)
        t = time.perf_counter()
        oracle.generic(u0, w["radius"], w["taps"], w["cids"], w["coef"], 1)
        one = time.perf_counter() - t
        k = max(1, min(200, int(20.0 / max(one, 1e-3))))
        t = time.perf_counter()
        oracle.generic(u0, w["radius"], w["taps"], w["cids"], w["coef"], k)
        dt = time.perf_counter() - t
        ac = all_cores(lambda: oracle.generic(u0, w["radius"], w["taps"], w["cids"], w["coef"], 1), 64 ** 3, one,
                       "1 sweep of the 64^3 crop")
        return dict(value=64 ** 3 * k / dt, unit="grid-point updates/s", cores=1, kind="oracle",
                    sample=f"64^3 crop of the same recipe, {k} sweeps, {dt:.1f} s, single thread", all_cores=ac)
    u0 = synth.heat3d7_input(96, 96, 96) if name == "heat3d7" else synth.heat2d5_input(256)
    cc = 0.4 if name == "heat3d7" else 0.6
    t = time.perf_counter()
    oracle.heat(u0, 20, cc, 0.1)
    one = time.perf_counter() - t
    k = max(20, min(200000, int(20 * 10.0 / max(one, 1e-4))))  # about 10 s of sweeps
    t = time.perf_counter()
    oracle.heat(u0, k, cc, 0.1)
    dt = time.perf_counter() - t
    pts = int(np.prod([s - 2 for s in u0.shape])) * k
    ac = all_cores(lambda: oracle.heat(u0, 20, cc, 0.1), int(np.prod([s - 2 for s in u0.shape])) * 20, one,
                   f"20 sweeps of the {u0.shape} padded grid")
    return dict(value=pts / dt, unit="grid-point updates/s", cores=1, kind="oracle",
                sample=f"{u0.shape} padded grid, {k} sweeps, {dt:.1f} s, single thread", all_cores=ac)


LHS_TILES = [(64, 4), (128, 2), (256, 1), (64, 8), (128, 4), (256, 2)]
PROGRAM_FORMS = ("plain", "cse", "cse_sat", "cse_bulk", "accsat", "accsat_z")


def program_ablation(torch, prog, n, host_ins, params, bytes_per_pt, reps=20):
    """A loop body through the saturator in the paper's ablation forms (and
    the z-streaming form): microseconds per out-of-place pass at each form's
    best launch shape (chosen first, from 5 timed passes per shape), then
    the mean of `reps` passes."""
    import concurrent.futures as cf

    from paper_2306_13002_amd import saturator as X

    ins = [torch.tensor(v, device="cuda") for v in host_ins]
    outs = [torch.zeros_like(ins[0]) for _ in range(prog["n_outputs"])]
    pts = n[0] * n[1] * n[2]
    tiles = [(64, 4), (128, 2), (256, 1), (32, 8), (64, 8)]
    shapes = {f: [(t[0], t[1], zb) for t in tiles for zb in ((16, 64, n[2]) if f == "accsat_z" else (1,))]
              for f in PROGRAM_FORMS}
    with cf.ThreadPoolExecutor(16) as ex:  # hipRTC compiles run in parallel
        plans = dict(ex.map(lambda ft: (ft, X.ProgramPlan(prog, n, ft[0], tile=ft[1][:2], zblock=ft[1][2])),
                            [(f, t) for f in PROGRAM_FORMS for t in shapes[f]]))

    def time_plan(pl, k):
        pl.profile(True)
        ms = []
        for _ in range(k):
            pl.run(ins, outs, params)
            ms.append(pl.profile_read())
        return ms

    res = {}
    try:
        for f in PROGRAM_FORMS:
            best = None
            for t in shapes[f]:
                time_plan(plans[(f, t)], 1)
                us = 1e3 * min(time_plan(plans[(f, t)], 5))
                if best is None or us < best[1]:
                    best = (t, us)
            ms = time_plan(plans[(f, best[0])], reps)
            us = 1e3 * sum(ms) / len(ms)
            st = X.generate(prog, n, f)[2]
            res[f] = {"us_per_sweep": us, "algorithmic_gbs": bytes_per_pt * pts / (us * 1e-6) / 1e9,
                      "tile": list(best[0]), "loads": st["loads"], "ops": st["ops"], "fmas": st["fmas"]}
    finally:
        for pl in plans.values():
            pl.close()
    return res


def bench_lhs(a, torch):
    """The saturator's lhs-assembly program: one step = one pass over the
    162^3 grid (75 outputs from 50 inputs, 1000 algorithmic bytes per point)."""
    import concurrent.futures as cf

    from paper_2306_13002_amd import saturator as X
    from paper_2306_13002_amd import synth

    n = synth.LHS_N
    prog = synth.lhs_program()
    host = synth.lhs_inputs(n)
    ins = [torch.tensor(v, device="cuda") for v in host]
    outs = [torch.zeros_like(ins[0]) for _ in range(75)]
    pts = n[0] * n[1] * n[2]
    bytes_per_pt = 8 * (50 + 75)
    forms = a.lhs_forms.split(",")
    tiles = [tuple(int(v) for v in a.lhs_tile.split(","))] if a.lhs_tile else LHS_TILES
    zbs = [int(v) for v in a.lhs_zblock.split(",")]

    def shapes(f):  # (tx, ty, z planes per thread): only the streaming form walks z (a z loop without
        # register windows measured slower for every form and block shape)
        return [(t[0], t[1], zb) for t in tiles for zb in (zbs if f == "accsat_z" else [1])]

    with cf.ThreadPoolExecutor(16) as ex:  # hipRTC compiles run in parallel
        plans = dict(ex.map(lambda ft: (ft, X.ProgramPlan(prog, n, ft[0], tile=ft[1][:2], zblock=ft[1][2])),
                            [(f, t) for f in forms for t in shapes(f)]))

    def time_plan(pl, k):
        pl.profile(True)
        ms = []
        for _ in range(k):
            pl.run(ins, outs, synth.LHS_PARAMS)
            ms.append(pl.profile_read())
        return ms

    res = {}
    for f in forms:
        best = None
        for t in shapes(f):  # launch shape per form, chosen before the timed region
            time_plan(plans[(f, t)], 2)
            us = 1e3 * min(time_plan(plans[(f, t)], 5))
            if best is None or us < best[1]:
                best = (t, us)
        pl = plans[(f, best[0])]
        # the wall clock with event profiling off, then the same steps profiled
        pl.profile(False)
        for _ in range(a.warmup):
            pl.run(ins, outs, synth.LHS_PARAMS)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            pl.run(ins, outs, synth.LHS_PARAMS)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = time_plan(pl, a.steps)
        launch = sum(ms) / len(ms) / 1e3
        res[f] = {"value": pts * a.steps / wall, "ms_per_step": wall * 1e3 / a.steps, "avg_launch_us": launch * 1e6,
                  "algorithmic_gbs": bytes_per_pt * pts / launch / 1e9, "tile": list(best[0]), **pl.info()}
    for p in plans.values():
        p.close()
    st = {f: X.generate(prog, n, f)[2] for f in forms}
    for f in forms:
        res[f].update(loads=st[f]["loads"], ops=st[f]["ops"], fmas=st[f]["fmas"], cost=st[f]["cost_extracted"])
        if "plain" in res:
            res[f]["over_plain"] = res[f]["value"] / res["plain"]["value"]
    sat_forms = [f for f in ("accsat", "accsat_z") if f in res] or [forms[-1]]
    main_form = max(sat_forms, key=lambda f: res[f]["value"])
    main_r = res[main_form]
    achieved = main_r["algorithmic_gbs"]
    traffic = read_traffic(f"lhs_{main_form}_162c", "saturator.cpp")
    out = {
        "metric": "grid-point updates/s (+ % of HBM peak), saturated vs plain",
        "value": main_r["value"], "unit": "grid-point updates/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": main_r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded recipe of the workload)",
        "config": {"workload": "block-tridiagonal assembly program, 162^3, 75 statements, 125 loads", "form": main_form,
                   "tile": main_r["tile"],
                   "launch_shape": "best of 6 block shapes (x 3 z-block depths for accsat_z) per form, before timing",
                   "interior": list(n), "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": f"sat_kernel_{main_form}", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": bytes_per_pt * pts, "avg_launch_us": main_r["avg_launch_us"]},
        "forms": res,
        "saturated_over_plain": main_r.get("over_plain"),
    }
    if not a.no_cpu:
        import oracle

        sub = [v[:6] for v in host]
        t = time.perf_counter()
        oracle.program(prog, sub, synth.LHS_PARAMS, (n[0], n[1], 4))
        one = time.perf_counter() - t
        k = max(4, min(160, int(4 * 20.0 / max(one, 1e-3))))
        sub = [v[:k + 2] for v in host]
        t = time.perf_counter()
        oracle.program(prog, sub, synth.LHS_PARAMS, (n[0], n[1], k))
        dt = time.perf_counter() - t
        out["cpu_baseline"] = {"value": n[0] * n[1] * k / dt, "unit": "grid-point updates/s", "cores": 1,
                               "kind": "oracle", "sample": f"{n[0]}x{n[1]}x{k} slab of the same recipe, {dt:.1f} s, "
                                                           "single thread"}
    print(json.dumps(out), flush=True)



METRIC = "grid-point updates/s + % HBM peak, saturated vs plain, at max rel err 1e-12 FP64"

# ---------------------------------------------------------------- wave25 headline
W25_N = (512, 512, 512)
W25_T = 10
# interior boxes [lo, hi) (x, y, z) compared with the oracle: a corner, the
# centre, and two boxes touching other faces and edges
W25_BOXES = [((0, 0, 0), (12, 9, 7)), ((250, 251, 249), (262, 259, 257)), ((500, 3, 505), (512, 11, 512)),
             ((100, 506, 0), (108, 512, 6))]


def maxrel(got, want) -> float:
    """max |got - want| / |want|; a nonzero value where want == 0 is infinite."""
    import numpy as np

    g = np.asarray(got, dtype=np.float64)
    w = np.asarray(want, dtype=np.float64)
    den = np.abs(w)
    if np.any((den == 0) & (g != 0)):
        return float("inf")
    den = np.where(den == 0, 1.0, den)
    return float(np.max(np.abs(g - w) / den)) if g.size else 0.0


def crop_slices(n, lo, hi, r, margin):
    """Padded-array slices (z, y, x) of a crop holding interior [lo, hi) plus
    `margin` interior cells per side (clipped at the real halo) and an r-wide
    halo, and the offsets of [lo, hi) inside the crop's interior.  After T
    leapfrog steps a point depends only on cells within 4T of it, and the
    two starting levels within 4(T-1), so a margin of 4(T-1) reproduces the
    full-grid values of [lo, hi) exactly."""
    sl, off = [], []
    for ax in range(3):
        a0 = max(lo[ax] - margin, 0)
        a1 = min(hi[ax] + margin, n[ax])
        sl.append(slice(a0, a1 + 2 * r))
        off.append((lo[ax] - a0, hi[ax] - a0))
    return tuple(reversed(sl)), tuple(reversed(off))


def region(lo, hi, r):
    """Padded-array slices (z, y, x) of interior [lo, hi)."""
    return tuple(slice(l + r, h + r) for l, h in reversed(list(zip(lo, hi))))


def timed(plan, step, reset, steps, warmup, torch):
    """W untimed steps, then K steps timed by the wall clock (synchronized on
    both sides) with the plan's event profiling off, then K more steps with
    it on, for the per-sweep kernel times: HIP events on the stream the
    sweeps are launched on.  (The events and their read-back add a few us per
    step, most of a step for the smallest workloads, so they stay out of the
    wall-clock region.)"""
    plan.profile(False)
    for _ in range(warmup):
        reset()
        step()
    reset()
    torch.cuda.synchronize()
    resid = None
    t0 = time.perf_counter()
    for _ in range(steps):
        resid = step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    plan.profile(True)
    sweep_ms, sweeps, per = 0.0, 0, []
    for _ in range(steps):
        step()
        ms, n = plan.profile_read()
        sweep_ms += ms
        sweeps += n
        per.append(ms / max(1, n))
    plan.profile(False)
    per.sort()
    return dict(wall=wall, sweep_ms=sweep_ms, sweeps=sweeps, resid=resid, sweep_ms_median=per[len(per) // 2],
                sweep_ms_best=per[0])


def host_info():
    """CPU model (lscpu, else /proc/cpuinfo) and core counts of this host."""
    import subprocess

    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    if not model:
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = None
    return {"cpu_model": model, "nproc": os.cpu_count(), "cores_available": aff}


def wave25_oracle_leg(a, b, v, gpu_regions, T):
    """The CPU-baseline leg of the headline: the oracle on the light-cone
    crops of the checked run (its outputs are compared with the GPU's) and on
    a 128^3 crop of the same recipe for about 10 s more, single thread, then
    the same crop calls on every core.  Returns (cpu_baseline, max rel err
    per form)."""
    import numpy as np

    import oracle
    from paper_2306_13002_amd import synth

    errs = {form: 0.0 for form in gpu_regions}
    pts = 0
    t0 = time.perf_counter()
    for bi, (lo, hi) in enumerate(W25_BOXES):
        sl, off = crop_slices(W25_N, lo, hi, 4, 4 * (T - 1))
        A, B, _ = oracle.wave25(a[sl], b[sl], v[sl], synth.WAVE25_COEF, T)
        pts += int(np.prod([s - 8 for s in A.shape])) * T
        cmp = tuple(slice(o0 + 4, o1 + 4) for o0, o1 in off)
        for form, regs in gpu_regions.items():
            ga, gb = regs[bi]
            errs[form] = max(errs[form], maxrel(ga, A[cmp]), maxrel(gb, B[cmp]))
    dt_crops = time.perf_counter() - t0
    c = 128
    ca, cb, cv = (x[:c + 8, :c + 8, :c + 8].copy() for x in (a, b, v))
    t = time.perf_counter()
    oracle.wave25(ca, cb, cv, synth.WAVE25_COEF, 1)
    one = time.perf_counter() - t
    k = max(1, min(200, int(10.0 / max(one, 1e-3))))
    t = time.perf_counter()
    oracle.wave25(ca, cb, cv, synth.WAVE25_COEF, k)
    dt = time.perf_counter() - t
    ac = all_cores(lambda: oracle.wave25(ca, cb, cv, synth.WAVE25_COEF, 2), c ** 3 * 2, 2 * one,
                   f"2 steps of the {c}^3 crop")
    total_pts = pts + c ** 3 * k
    cpu = dict(value=total_pts / (dt_crops + dt), unit="grid-point updates/s", cores=1, kind="oracle",
               sample=f"the oracle, single thread: {len(W25_BOXES)} light-cone crops of the checked 512^3 run "
                      f"({pts} updates, {dt_crops:.1f} s; compared with the GPU) and a {c}^3 crop of the same "
                      f"recipe for {k} steps ({c ** 3 * k} updates, {dt:.1f} s)",
               host=host_info(), all_cores=ac)
    return cpu, errs


def wave25_headline(a, torch, synth, Plan, dev):
    """The metric's configuration: saturated and plain wave25 at 512^3."""
    import numpy as np

    T = W25_T
    pts_step = W25_N[0] * W25_N[1] * W25_N[2] * T
    ha, hb, hv = synth.wave25_inputs(W25_N[0])
    f = [torch.empty(ha.shape, dtype=torch.float64, device=dev) for _ in range(2)]
    vs = torch.tensor(hv, device=dev)
    src = [torch.tensor(ha, device=dev), torch.tensor(hb, device=dev)]  # the seeded start, kept on the device
    forms = ["saturated"] if a.no_plain else ["saturated", "plain"]
    res, regions, resid_check = {}, {}, {}
    for form in forms:
        print(f"[bench] wave25 {form}: plan (tuning)", file=sys.stderr, flush=True)
        plan = Plan("wave25", W25_N, variant=form, coef=synth.WAVE25_COEF, tune=TUNE)
        print(f"[bench] wave25 {form}: {plan.config()}; checked run, then timing", file=sys.stderr, flush=True)
        # the checked run: T steps from the seeded start at the timed launch shape
        for i in range(2):
            f[i].copy_(src[i])
        plan.run(f, [vs], iterations=T)
        gr = plan.residual()
        regions[form] = [(f[0][region(lo, hi, 4)].cpu().numpy(), f[1][region(lo, hi, 4)].cpu().numpy())
                         for lo, hi in W25_BOXES]
        # the residual against the returned fields (on the device, FP64): the
        # two-pass reduction at the benchmarked size
        newest, older = (f[0], f[1]) if T % 2 == 1 else (f[1], f[0])
        d = newest[4:-4, 4:-4, 4:-4] - older[4:-4, 4:-4, 4:-4]
        rs = float((d * d).sum())
        del d
        resid_check[form] = {"library": gr, "from_fields": rs, "rel_err": abs(gr - rs) / rs}

        def step(plan=plan):
            plan.run(f, [vs], iterations=T)
            return plan.residual()

        r = timed(plan, step, lambda: None, a.steps, a.warmup, torch)
        r["cfg"] = plan.config()
        res[form] = r
        if form == "plain" and not a.no_ablation:
            # the paper's ablation forms (per point), at the plain form's tuned shape
            abl = {}
            for v in ("cse_sat", "cse_bulk", "accsat_point"):
                with Plan("wave25", W25_N, variant=v, coef=synth.WAVE25_COEF, tile=tuple(r["cfg"]["tile"])) as pv:
                    ra = timed(pv, lambda pv=pv: (pv.run(f, [vs], iterations=T), pv.residual())[1], lambda: None,
                               max(2, a.steps // 4), 1, torch)
                abl[v] = {"us_per_sweep": ra["sweep_ms"] * 1e3 / max(1, ra["sweeps"])}
            res["ablation"] = abl
        plan.close()
    del src, f, vs
    torch.cuda.empty_cache()
    sat = res["saturated"]
    launch_s = sat["sweep_ms"] / 1e3 / max(1, sat["sweeps"])
    alg = 32.0 * W25_N[0] * W25_N[1] * W25_N[2]
    achieved = alg / launch_s / 1e9
    traffic = read_traffic("wave25_sat_512c", ("wave25.hip", "common.hpp"))
    tx, ty, zb = sat["cfg"]["tile"]
    value = pts_step * a.steps / sat["wall"]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "grid-point updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": sat["wall"] * 1e3 / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded recipe: v ~ U[1.5,4.5), vsq = (0.4 v/4.5)^2, u^-1 = u^0 = 1 + 0.1 U[0,1))",
        "config": {
            "workload": "wave25 radius-4 25-point leapfrog, FP64, 512x512x512 interior + 4-cell halo, 10 steps "
                        "per benchmark step + FP64 residual",
            "variant": "saturated", "tile": [tx, ty, zb], "tile_map": sat["cfg"].get("tile_map"),
            "launch_shape": "autotuned (exhaustive, at plan time)", "interior": list(W25_N),
            "iterations_per_step": T, "storage": "f64", "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm", "kernel": f"wave25_sat tile {tx}x{ty}, zblock {zb}", "achieved": achieved,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "algorithmic_bytes_per_launch": alg, "bytes_per_update": 32, "updates_per_launch": alg / 32,
            "avg_launch_us": launch_s * 1e6, "median_launch_us": sat["sweep_ms_median"] * 1e3,
            "best_launch_us": sat["sweep_ms_best"] * 1e3,
            "traffic_gbs": traffic / launch_s / 1e9 if traffic else None,
            "traffic_over_algorithmic": traffic / alg if traffic else None,
            "timing": "HIP events on the launch stream around the timed steps' sweep launches",
        },
        "residual": sat["resid"],
        "residual_check": resid_check,
    }
    if "plain" in res:
        pr = res["plain"]
        pl = pr["sweep_ms"] / 1e3 / max(1, pr["sweeps"])
        pv = pts_step * a.steps / pr["wall"]
        out["plain"] = {"value": pv, "ms_per_step": pr["wall"] * 1e3 / a.steps, "avg_launch_us": pl * 1e6,
                        "achieved_gbs": alg / pl / 1e9, "frac": alg / pl / 1e9 / HBM_PEAK_GBS,
                        "tile": list(pr["cfg"]["tile"]),
                        "traffic": read_traffic("wave25_plain_512c", ("wave25.hip", "common.hpp"))}
        out["saturated_over_plain"] = value / pv
        if "ablation" in res:
            abl = {"plain": {"us_per_sweep": pl * 1e6}, **res["ablation"],
                   "saturated": {"us_per_sweep": launch_s * 1e6}}
            for v in abl.values():
                v["algorithmic_gbs"] = alg / (v["us_per_sweep"] * 1e-6) / 1e9
            out["ablation"] = abl
    tol = {"saturated": 1e-12, "plain": 0.0}
    if not a.no_cpu:
        print("[bench] oracle leg (light-cone crops, CPU baseline)", file=sys.stderr, flush=True)
        cpu, errs = wave25_oracle_leg(ha, hb, hv, regions, T)
        out["cpu_baseline"] = cpu
        ok = all(errs[k] <= tol[k] for k in errs) and all(c["rel_err"] <= 1e-10 for c in resid_check.values())
        out["parity"] = {"oracle": f"CPU FP64 oracle on {len(W25_BOXES)} light-cone crops of the same 512^3 run "
                                   "(corner, centre, faces and edges), both time levels",
                         "max_rel_err": errs, "tolerance": tol, "residual_tolerance": 1e-10, "pass": ok}
    else:
        out["parity"] = {"pass": None, "note": "not checked (--no-cpu skips the oracle leg)"}
    return out


# ---------------------------------------------------------------- streaming ceilings
STREAM_VARIANTS = [  # (op, width, nt_loads, nt_stores, in_place)
    ("3r1w", 1, False, False, True), ("3r1w", 2, False, False, True), ("3r1w", 1, True, True, True),
    ("3r1w", 2, True, True, True), ("3r1w", 1, False, True, True), ("3r1w", 2, False, True, True),
    ("3r1w", 1, False, False, False), ("copy", 1, False, False, False), ("copy", 2, False, False, False),
    ("copy", 2, True, True, False),
]


def stream_ceilings(torch, dev, reps=10, edge=520):
    """HBM ceilings of the sweeps' access shapes with the library's streaming
    kernels on edge^3 FP64 arrays (the wave25 grid's storage): three reads +
    one write in place (the leapfrog step), and copies (the Jacobi sweeps);
    best and median of `reps` launches, HIP events on the launch stream."""
    from paper_2306_13002_amd.stencil import stream

    n = edge ** 3
    A = torch.full((n,), 1.0, dtype=torch.float64, device=dev)
    B = torch.full((n,), 0.5, dtype=torch.float64, device=dev)
    C = torch.full((n,), 0.25, dtype=torch.float64, device=dev)
    D = torch.empty(n, dtype=torch.float64, device=dev)
    out = {}
    for op, w, ntl, nts, inplace in STREAM_VARIANTS:
        d = B if (op == "3r1w" and inplace) else D
        bb, cc = (B, C) if op == "3r1w" else (None, None)
        ms = []
        for i in range(reps + 2):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            stream(op, A, bb, cc, d, width=w, nt_loads=ntl, nt_stores=nts)
            e1.record()
            e1.synchronize()
            if i >= 2:
                ms.append(e0.elapsed_time(e1))
        if op == "3r1w" and inplace:
            B.fill_(0.5)
        ms.sort()
        nbytes = (32 if op == "3r1w" else 16) * n
        name = f"{op}{'_inplace' if inplace else ''}_w{w}{'_ntload' if ntl else ''}{'_ntstore' if nts else ''}"
        out[name] = {"bytes": nbytes, "best_us": ms[0] * 1e3, "median_us": ms[len(ms) // 2] * 1e3,
                     "best_gbs": nbytes / (ms[0] * 1e-3) / 1e9, "median_gbs": nbytes / (ms[len(ms) // 2] * 1e-3) / 1e9}
    del A, B, C, D
    torch.cuda.empty_cache()
    return {"arrays": f"{edge}^3 FP64 ({n * 8 / 2 ** 30:.3f} GiB each)", "kernel": "stencil_stream (stream.hip)",
            "variants": out}


# ---------------------------------------------------------------- secondary workloads
def secondary_jacobi(name, a, dev, torch, synth, Plan):
    """poisson19 129x129x257 or heat3d7 160^3: every form, tuned; per-pass and
    per-sweep-equivalent fractions kept apart; cache residency flagged."""
    forms = ["plain", "saturated", "saturated_t2"] + (["saturated_t3"] if name == "heat3d7" else [])
    steps = max(5, a.steps // 2)
    rows = {}
    meta = None
    for v in forms:
        r = time_variant(name, v, steps, 2, dev, torch, synth, Plan)
        meta = r["meta"]
        per_launch = meta.get("sweeps_per_launch", 1)
        sweep_s = r["sweep_ms"] / 1e3 / max(1, r["sweeps"])
        launch_s = sweep_s * per_launch
        pts_sweep = r["pts"] / r["T"]
        alg = meta["bytes_per_update"] * pts_sweep
        traffic = read_traffic(meta["kernel_tag"], meta["source"])
        rows[v] = {"us_per_sweep": sweep_s * 1e6, "avg_launch_us": launch_s * 1e6, "sweeps_per_launch": per_launch,
                   "tile": list(r["cfg"]["tile"]), "tile_map": r["cfg"].get("tile_map"),
                   "updates_per_s": r["pts"] * steps / r["wall"],
                   "frac_per_pass": alg / launch_s / 1e9 / HBM_PEAK_GBS,
                   "frac_sweep_equivalent": alg * per_launch / launch_s / 1e9 / HBM_PEAK_GBS,
                   "traffic_per_launch": traffic, "traffic_gbs": traffic / launch_s / 1e9 if traffic else None}
    n_arrays = 14 if name == "poisson19" else 2
    ws = n_arrays * (4 if meta["storage"] == "f32" else 8)
    pts_total = 1
    for e in (meta.get("grid_total") or [x + 2 for x in meta["interior"]]):
        pts_total *= e
    ws *= pts_total
    out = {
        "workload": meta["workload"], "storage": meta["storage"], "working_set_bytes": ws,
        "cache_resident": ws <= INFINITY_CACHE_BYTES,
        "note": ("working set fits the 256 MB Infinity Cache: rates above are cache-assisted, not an HBM roofline"
                 if ws <= INFINITY_CACHE_BYTES else "working set exceeds the Infinity Cache"),
        "forms": rows,
        # the paper's per-point rewrites vs. temporal blocking (two sweeps per pass, not in the paper)
        "rewrite_gain_saturated_over_plain": rows["plain"]["us_per_sweep"] / rows["saturated"]["us_per_sweep"],
        "temporal_blocking_gain_t2_over_saturated":
            rows["saturated"]["us_per_sweep"] / rows["saturated_t2"]["us_per_sweep"],
    }
    if "saturated_t3" in rows:  # three sweeps per pass (heat3d7)
        out["temporal_blocking_gain_t3_over_saturated"] = (rows["saturated"]["us_per_sweep"] /
                                                           rows["saturated_t3"]["us_per_sweep"])
    return out


def secondary_batch(a, dev, torch, synth, Plan):
    steps = max(3, a.steps // 4)
    rows = {}
    for v in ("saturated_t2", "saturated_t3", "plain"):
        r = time_variant("batch", v, steps, 1, dev, torch, synth, Plan)
        rows[v] = {"us_per_iteration": r["sweep_ms"] * 1e3 / max(1, r["sweeps"]),
                   "updates_per_s": r["pts"] * steps / r["wall"], "ms_per_step": r["wall"] * 1e3 / steps}
        if "classes" in r["cfg"]:
            rows[v]["classes"] = [{"variant": c["variant"], "tile": list(c["tile"]), "problems": c["problems"]}
                                  for c in r["cfg"]["classes"]]
        pts = r["pts"] // r["T"]
    alg = 16.0 * pts
    for v in rows.values():
        v["frac_per_sweep"] = alg / (v["us_per_iteration"] * 1e-6) / 1e9 / HBM_PEAK_GBS
    return {"workload": "64 independent heat3d7 FP64 grids, edges 32..160 (seeded), 50 sweeps each + residuals",
            "updates_per_iteration": pts, "working_set_bytes": 16 * pts,
            "forms": {"batched_graph_two_sweep": rows["saturated_t2"], "batched_graph_three_sweep": rows["saturated_t3"],
                      "separate_plain_runs": rows["plain"]},
            "batched_over_separate": rows["plain"]["us_per_iteration"] /
                                     min(rows["saturated_t2"]["us_per_iteration"],
                                         rows["saturated_t3"]["us_per_iteration"])}


def secondary_heat2d5(a, dev, torch, synth, Plan):
    """heat2d5 256^2, 10 sweeps + residual per step (the plain form only): one
    launch per sweep and sweeps fused per launch (tuned), and the oracle on
    one core and on every core at once (each thread its own grid)."""
    steps = max(50, 5 * a.steps)
    rows, meta = {}, None
    for label, kw in (("one_launch_per_sweep", dict(tile=(64, 8, 1))), ("fused_tuned", {})):
        r = time_variant("heat2d5", "plain", steps, 5, dev, torch, synth, Plan, plan_kw=kw)
        meta = r["meta"]
        rows[label] = {"updates_per_s": r["pts"] * steps / r["wall"], "us_per_step": r["wall"] * 1e6 / steps,
                       "tile": list(r["cfg"]["tile"])}
    out = {"workload": meta["workload"], "forms": rows,
           "fused_over_one_launch_per_sweep": rows["fused_tuned"]["updates_per_s"] /
           rows["one_launch_per_sweep"]["updates_per_s"]}
    if not a.no_cpu:
        cb = cpu_baseline("heat2d5")
        out["cpu_baseline"] = cb
        out["gpu_over_cpu_all_cores"] = rows["fused_tuned"]["updates_per_s"] / cb["all_cores"]["value"]
    return out


def run_secondary(out, a, dev, torch, synth, Plan):
    sec = {}
    for key, fn in (("stream", lambda: stream_ceilings(torch, dev)),
                    ("poisson19", lambda: secondary_jacobi("poisson19", a, dev, torch, synth, Plan)),
                    ("heat3d7", lambda: secondary_jacobi("heat3d7", a, dev, torch, synth, Plan)),
                    ("batch", lambda: secondary_batch(a, dev, torch, synth, Plan)),
                    ("heat2d5", lambda: secondary_heat2d5(a, dev, torch, synth, Plan))):
        try:
            sec[key] = fn()
        except Exception as e:  # a secondary failure must not hide the headline
            sec[key] = {"error": f"{type(e).__name__}: {e}"}
        print(f"[bench] secondary {key} done", file=sys.stderr, flush=True)
    out["secondary"] = sec
    if "stream" in sec and "variants" in sec["stream"]:
        v = sec["stream"]["variants"]
        best = max(x["best_gbs"] for k, x in v.items() if k.startswith("3r1w_inplace"))
        out["roofline"]["stream_ceiling_3r1w_gbs"] = best
        out["roofline"]["frac_of_stream_ceiling"] = out["roofline"]["achieved"] / best


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="wave25",
                    choices=["wave25", "poisson19", "heat2d5", "heat3d7", "batch", "copy", "lhs", "generic", "stream"])
    ap.add_argument("--variant", default="best", choices=["best", "saturated", "saturated_t2", "saturated_t3", "plain"],
                    help="non-headline workloads: best = every saturated form the workload offers, tuned, the "
                         "fastest reported")
    ap.add_argument("--no-plain", action="store_true", help="skip timing the plain form beside it")
    ap.add_argument("--no-ablation", action="store_true", help="wave25: skip the per-point ablation forms")
    ap.add_argument("--no-secondary", action="store_true", help="wave25: only the headline, no secondary objects")
    ap.add_argument("--lhs-forms", default="plain,cse,cse_sat,cse_bulk,accsat,accsat_z",
                    help="lhs workload: the saturator forms to time")
    ap.add_argument("--lhs-zblock", default="8,16,32", help="lhs workload: z planes per thread tried for accsat_z")
    ap.add_argument("--lhs-tile", default="", help="lhs workload: one block shape 'tx,ty' instead of the search")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg (and with it the oracle parity)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {a.gpus} requested); the stencil library has no "
              "multi-GPU path in this build", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2306_13002_amd import synth
    from paper_2306_13002_amd.stencil import Plan

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if a.workload == "lhs":
        return bench_lhs(a, torch)
    if a.workload == "stream":
        print(json.dumps({"metric": "HBM streaming ceiling (GB/s) of the sweeps' access shapes",
                          "stream": stream_ceilings(torch, dev, reps=max(3, a.steps))}), flush=True)
        return
    if a.workload == "wave25" and a.variant in ("best", "saturated"):
        out = wave25_headline(a, torch, synth, Plan, dev)
        print("[bench] headline done", file=sys.stderr, flush=True)
        if not a.no_secondary:
            run_secondary(out, a, dev, torch, synth, Plan)
        print(json.dumps(out), flush=True)
        if out["parity"]["pass"] is False:
            print("[bench] PARITY FAILURE against the oracle", file=sys.stderr, flush=True)
            sys.exit(1)
        return
    bench_workload(a, dev, torch, synth, Plan)


def bench_workload(a, dev, torch, synth, Plan):
    """One workload alone (profiling runs): its saturated forms, the plain
    form beside them, the oracle's CPU rate."""
    forms = [a.variant]
    if a.variant == "best":
        forms = ["saturated", "saturated_t2"] if a.workload in ("poisson19", "heat3d7", "batch") else ["saturated"]
        if a.workload in ("heat3d7", "batch"):  # three sweeps per pass: heat3d7 only
            forms.append("saturated_t3")
        if a.workload == "heat2d5":  # the 2-D heat sweep has the plain form only
            forms = ["plain"]
    sat = {v: time_variant(a.workload, v, a.steps, a.warmup, dev, torch, synth, Plan) for v in forms}
    variant = max(forms, key=lambda v: sat[v]["pts"] / sat[v]["wall"])
    main_r = sat[variant]
    meta = main_r["meta"]
    value = main_r["pts"] * a.steps / main_r["wall"]
    ms_per_step = main_r["wall"] * 1000.0 / a.steps
    sweep_s = main_r["sweep_ms"] / 1000.0 / max(1, main_r["sweeps"])
    per_launch = meta.get("sweeps_per_launch", 1)
    launch_s = sweep_s * per_launch
    pts_per_sweep = main_r["pts"] / main_r["T"]
    alg_bytes = meta["bytes_per_update"] * pts_per_sweep  # one pass over the grid per launch
    achieved = alg_bytes / launch_s / 1e9
    traffic = read_traffic(meta["kernel_tag"], meta["source"])
    roof = {
        "bound": "hbm",
        "kernel": meta["kernel_tag"],
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        "traffic": traffic,
        "algorithmic_bytes_per_launch": alg_bytes,
    }
    if meta.get("bound") == "alu":
        # FP64 vector peak: 256 CUs x 2.4 GHz x 128 FP64 flops per clock (64 FMA lanes) = 78.6 TFLOP/s, i.e.
        # 39.3e12 FP64 instructions/s (an add issues like an FMA but counts one flop)
        fl = meta["flops_per_update"] * pts_per_sweep / launch_s / 1e12
        ins = meta["instr_per_update"] * pts_per_sweep / launch_s
        roof = {"bound": "alu", "kernel": meta["kernel_tag"], "achieved": fl, "peak": FP64_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": fl / FP64_VECTOR_PEAK_TFLOPS, "traffic": traffic,
                "algorithmic_flops_per_launch": meta["flops_per_update"] * pts_per_sweep,
                "fp64_instr_per_s": ins, "issue_frac": ins / (FP64_VECTOR_PEAK_TFLOPS * 1e12 / 2),
                "hbm_gbs": alg_bytes / launch_s / 1e9}
    out = {
        "metric": METRIC if meta["storage"] == "f64" else "grid-point updates/s (+ % of HBM peak), saturated vs plain",
        "value": value,
        "unit": "grid-point updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": meta["storage"],
        "arithmetic": "f64",
        "data": "synthetic (seeded recipe of the workload)",
        "config": {
            "workload": meta["workload"],
            "variant": variant,
            "sweeps_per_launch": per_launch,
            "tile": list(main_r["cfg"]["tile"]),
            "tile_map": main_r["cfg"].get("tile_map"),
            "launch_shape": "autotuned (exhaustive, plan time)",
            "interior": meta["interior"],
            "iterations_per_step": meta["iterations"],
            "storage": meta["storage"],
            "parallelism": "single GPU",
        },
        "roofline": {
            **roof,
            "avg_launch_us": launch_s * 1e6,
            "median_launch_us": main_r["sweep_ms_median"] * 1e3 * per_launch,
            "best_launch_us": main_r["sweep_ms_best"] * 1e3 * per_launch,
            "traffic_gbs": traffic / launch_s / 1e9 if traffic else None,
        },
        "residual": main_r["resid"],
    }
    if "classes" in main_r["cfg"]:  # batched plans: one form and launch shape per size class
        out["config"]["classes"] = [{"variant": c["variant"], "tile": list(c["tile"]), "problems": c["problems"]}
                                    for c in main_r["cfg"]["classes"]]
    if per_launch > 1 and roof["bound"] == "hbm":
        # a launch advances per_launch sweeps for one pass of bytes: the rate a
        # single-sweep kernel would need to match it (may exceed the peak)
        out["roofline"]["sweep_equivalent"] = {"achieved": achieved * per_launch,
                                               "frac": achieved * per_launch / HBM_PEAK_GBS}
    if len(forms) > 1:
        out["saturated_forms"] = {
            v: {"value": r["pts"] * a.steps / r["wall"], "us_per_sweep": r["sweep_ms"] * 1e3 / max(1, r["sweeps"]),
                "sweeps_per_launch": r["meta"].get("sweeps_per_launch", 1), "tile": list(r["cfg"]["tile"]),
                "tile_map": r["cfg"].get("tile_map")} for v, r in sat.items()}
    if not a.no_plain and variant != "plain" and a.workload not in ("heat2d5", "copy"):
        pr = time_variant(a.workload, "plain", a.steps, a.warmup, dev, torch, synth, Plan)
        pv = pr["pts"] * a.steps / pr["wall"]
        pl = pr["sweep_ms"] / 1000.0 / max(1, pr["sweeps"])
        out["plain"] = {"value": pv, "ms_per_step": pr["wall"] * 1000.0 / a.steps, "us_per_sweep": pl * 1e6,
                        "achieved_gbs": meta["bytes_per_update"] * pts_per_sweep / pl / 1e9, "avg_launch_us": pl * 1e6,
                        "tile": list(pr["cfg"]["tile"]), "tile_map": pr["cfg"].get("tile_map")}
        out["saturated_over_plain"] = value / pv
        if a.workload == "poisson19" and "saturated" in sat:
            # the paper's ablation forms (per point), at the plain form's tuned shape
            abl = {"plain": {"us_per_sweep": pl * 1e6},
                   "saturated": {"us_per_sweep": sat["saturated"]["sweep_ms"] * 1e3 / max(1, sat["saturated"]["sweeps"])}}
            for form in ("cse_sat", "cse_bulk", "accsat_point"):
                fr = time_variant(a.workload, form, max(2, a.steps // 4), 2, dev, torch, synth, Plan,
                                  dict(tune="fixed", tile=tuple(pr["cfg"]["tile"])))
                abl[form] = {"us_per_sweep": fr["sweep_ms"] / 1000.0 / max(1, fr["sweeps"]) * 1e6}
            for v in abl.values():
                v["algorithmic_gbs"] = meta["bytes_per_update"] * pts_per_sweep / (v["us_per_sweep"] * 1e-6) / 1e9
            out["ablation"] = abl
        if a.workload == "heat3d7":
            # the loop body through the saturator (generated kernels, one pass per launch) in the paper's
            # ablation forms, beside the hand-written kernels' single-sweep forms
            n3 = tuple(meta["interior"])
            abl = program_ablation(torch, synth.heat3d7_program(), n3, [synth.heat3d7_input(*n3)], [0.4, 0.1],
                                   meta["bytes_per_update"])
            abl["kernel_plain"] = {"us_per_sweep": pl * 1e6}
            if "saturated" in sat:
                abl["kernel_saturated"] = {"us_per_sweep": sat["saturated"]["sweep_ms"] * 1e3 /
                                           max(1, sat["saturated"]["sweeps"])}
            out["ablation"] = abl
    if not a.no_cpu and a.workload not in ("copy", "batch"):
        out["cpu_baseline"] = cpu_baseline(a.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
