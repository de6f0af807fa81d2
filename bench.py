"""Throughput of the fused DUGKS step on one MI355X.

Workload (the headline configuration): one D2Q9 DUGKS T2 step of the
conservative Allen-Cahn equation on a 4096 x 4096 periodic grid, upwind-3
(third-order isotropic) reconstruction, W = 4, M = 0.01, C = 0.5, 64 random
tanh circles (R 20-200 cells, seed 0) in rigid rotation (corner speed 0.05).
State is resident in HBM before the timed region.  The tile height of each
plain-path run is the one recorded with the committed PMC summary of the same
kernel sources (the autotuner's earlier pick), else measured on that state
first (dugks_tune; the state is left unchanged).  The timed region is exactly --steps calls of the step (one fused
kernel each).  FP64 is the headline line;
the FP32 form (FP32 storage, FP64 mass sums and the fused mass correction on
every step) is reported in the same line, and so are the batched form (256
uneven grids, 32-512 per side, one persistent kernel, hipGraph replays of 50
steps, autotuned tile height, against one launch per grid and step) and the
serving form (a scaled request stream served by continuous batching, against
one-at-a-time execution), and the three-level DUGKS-T3S3 step (two fused
stage kernels per step) on the same field with M = 0.02, since T3S3 needs
dt < 12 tau = 36 M.

MLUPS = nx * ny * steps / time / 1e6.  Algorithmic traffic per lattice update:
f~^n in and f~^{n+1} out (9 + 9 words), phi^{n-1} in and phi^n out (2 words):
160 B in FP64, 80 B in FP32.  T3S3: stage A reads f^^n and phi^{n-1} (10
words) and writes f~(t') with the phi plane and Q (19), stage B reads both
(19) and writes f^^{n+1} (10): 58 words, 464 B in FP64.  Peak HBM bandwidth of
MI355X: 8 TB/s.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HBM_PEAK_GBS = 8000.0
WORDS_PER_LU = 20
WORDS_PER_LU_T3S3 = 58
T3S3_MOBILITY = 0.02
# stated targets: the 4096^2 upwind-3 step at >= 70 % of the HBM peak; the FP32
# form within 1e-5 relative L2 of phi and 1e-9 relative mass drift
TARGET_FRAC = 0.70
TARGET_FP32_L2 = 1e-5
TARGET_FP32_DRIFT = 1e-9
CPU_STEPS = 16         # oracle sample of the headline grid: about 10-20 s on the host cores
# steps run before any timed region whatever --warmup says: the GPU's clocks
# ramp up over the first ~20 steps after idle (690 -> 636 us per FP64 step)
CLOCK_WARMUP_STEPS = 50


def progress(msg):
    """One line per finished leg on stderr (stdout carries only the JSON line)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--size", type=int, default=4096)
    ap.add_argument("--tile-rows", type=int, default=0,
                    help="tile height of the plain FP64 run (0: autotuned with dugks_tune)")
    ap.add_argument("--tile-rows-f32", type=int, default=0,
                    help="tile height of the plain FP32 run (0: autotuned)")
    ap.add_argument("--tile-rows-t3s3", type=int, default=0,
                    help="tile height of the T3S3 run (0: autotuned)")
    ap.add_argument("--batch-steps", type=int, default=2000)
    ap.add_argument("--serve-requests", type=int, default=64)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--batch-kernel-rows", type=int, default=0,
                    help="only the batch kernel on the C4 grids at this tile height, "
                         "--batch-steps plain launches (counter runs)")
    ap.add_argument("--only-batch", action="store_true",
                    help="the batched section alone (profiling runs)")
    ap.add_argument("--no-t3s3", action="store_true")
    ap.add_argument("--no-t2s5", action="store_true")
    ap.add_argument("--no-shard", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", choices=["f64", "f32"], default=None,
                    help="time one precision only (profiling runs)")
    return ap.parse_args()


def time_steps(solver, steps, warmup):
    """Warm up (CLOCK_WARMUP_STEPS, then `warmup` more), then time exactly
    `steps` steps with HIP events on the stream the kernels run on; returns
    (seconds, ms of the timed region)."""
    import torch
    for k in range(CLOCK_WARMUP_STEPS + warmup):
        solver.step(1)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(stream)
    for k in range(steps):
        solver.step(1)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = start.elapsed_time(stop)
    return wall, ev_ms


def time_kernel_only(solver, steps):
    """Mean duration of the fused step kernel alone (HIP events around a run
    of back-to-back launches on the same stream)."""
    import torch
    stream = torch.cuda.current_stream()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    solver.step(steps)
    stop.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / steps


def copy_bandwidth():
    """Read+write bandwidth of a plain streaming kernel (an elementwise scale of
    1 GiB into 1 GiB), GB/s.  The same kernel calibrates the PMC byte counters:
    it moves exactly 2 GiB per launch."""
    import torch
    n = 1 << 30   # bytes per side
    a = torch.empty(n // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        torch.mul(a, 1.000001, out=b)
    torch.cuda.synchronize()
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    s.record()
    reps = 10
    for _ in range(reps):
        torch.mul(a, 1.000001, out=b)
    e.record()
    torch.cuda.synchronize()
    gbs = 2 * n * reps / (s.elapsed_time(e) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs


def _profile_record(name: str, tile_rows: int):
    """A committed rocprofv3 PMC summary (profiles/<name>.json) if it was taken
    with the current kernel sources and the same tile height (the halo
    rows re-read depend on it), else None."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", name + ".json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
        from paper_2007_07760_amd import kernel_fingerprint
        if rec.get("kernel_fingerprint") != kernel_fingerprint():
            return None
        if rec.get("tile_rows") != tile_rows:
            return None
        return rec
    except Exception:
        return None


def profiled_tile_rows(name: str):
    """The tile height a committed PMC summary was taken at, when it matches
    the current kernel sources: the autotuner's pick for this kernel
    version, reused (a tuning cache), so that the run and its traffic figure
    describe the same launches.  None: tune."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", name + ".json")
    try:
        rec = json.load(open(path))
        from paper_2007_07760_amd import kernel_fingerprint
        if rec.get("kernel_fingerprint") == kernel_fingerprint():
            return int(rec["tile_rows"])
    except Exception:
        pass
    return None


def pick_tile(solver, given: int, profile: str):
    """(rows, source): the given height, else the profiled one, else tuned."""
    if given:
        return given, "given"
    rows = profiled_tile_rows(profile)
    if rows:
        solver.retile(rows)
        return rows, "profiled"
    return solver.tune(), "tuned"


def profile_traffic(precision: str, tile_rows: int):
    """HBM bytes per launch of the T2 step kernel (profiles/traffic_h1_<precision>.json)."""
    rec = _profile_record(f"traffic_h1_{precision}", tile_rows)
    return rec.get("bytes_per_launch") if rec else None


def profile_traffic_t3s3(tile_rows: int):
    """HBM bytes of one T3S3 step (stage A + stage B launches)."""
    rec = _profile_record("traffic_h1_t3s3_f64", tile_rows)
    if not rec:
        return None
    return rec["stage_a"]["bytes_per_launch"] + rec["stage_b"]["bytes_per_launch"]


def bench_t3s3(w, steps, warmup, tile_rows):
    """The DUGKS-T3S3 step (stage A + stage B kernels) on the headline field
    with M = T3S3_MOBILITY, FP64."""
    import torch
    from paper_2007_07760_amd import _lib as C
    from paper_2007_07760_amd.solver import Solver
    s = Solver(w["nx"], w["ny"], T3S3_MOBILITY, w["width"], w["cfl"], recon=w["recon"],
               precision=C.F64, vel_kind=w["vel_kind"], vel_param=w["vel_param"],
               scheme=C.T3S3, tile_rows=tile_rows).init(w["phi0"])
    rows, source = pick_tile(s, tile_rows, "traffic_h1_t3s3_f64")
    wall, ev_ms = time_steps(s, steps, warmup)
    k_ms = time_kernel_only(s, min(steps, 50))
    lus = w["nx"] * w["ny"]
    achieved = WORDS_PER_LU_T3S3 * 8 * lus / (k_ms * 1e-3) / 1e9
    del s
    torch.cuda.empty_cache()
    # the FP32 form of the same step, with the fused mass correction
    s = Solver(w["nx"], w["ny"], T3S3_MOBILITY, w["width"], w["cfl"], recon=w["recon"],
               precision=C.F32, vel_kind=w["vel_kind"], vel_param=w["vel_param"],
               flags=C.FLAG_MASS_FIX, scheme=C.T3S3).init(w["phi0"])
    rows32, source32 = s.tune(), "tuned"
    _, ev32 = time_steps(s, steps, warmup)
    m0 = s.mass0()
    drift = abs(s.mass() - m0) / m0
    del s
    torch.cuda.empty_cache()
    return {"value": round(lus * steps / (ev_ms * 1e-3) / 1e6, 1), "unit": "MLUPS",
            "ms_per_step": round(ev_ms / steps, 4), "dtype": "f64",
            "mobility": T3S3_MOBILITY, "kernels": "step_kernel stage A + stage B",
            "step_kernels_ms": round(k_ms, 4), "achieved": round(achieved, 1),
            "frac": round(achieved / HBM_PEAK_GBS, 4), "tile_rows": rows, "tile_source": source,
            "traffic": profile_traffic_t3s3(rows), "bytes_per_lu": WORDS_PER_LU_T3S3 * 8,
            "fp32": {"value": round(lus * steps / (ev32 * 1e-3) / 1e6, 1), "unit": "MLUPS",
                     "ms_per_step": round(ev32 / steps, 4), "dtype": "f32",
                     "mass_correction": "fused, every step",
                     "relative_mass_drift": float(f"{drift:.3g}"), "tile_rows": rows32,
                     "tile_source": source32, "bytes_per_lu": WORDS_PER_LU_T3S3 * 4}}


def bench_t2s5(w, steps, warmup):
    """DUGKS-T2S5 (the fifth-order reconstruction, one fused kernel per step
    like T2S3) on the headline field, FP64 and FP32 with the fused mass
    correction; the same 160 / 80 B of algorithmic traffic per update."""
    import torch
    from paper_2007_07760_amd import _lib as C
    from paper_2007_07760_amd.solver import Solver
    out = {}
    lus = w["nx"] * w["ny"]
    for name, prec, flags in (("f64", C.F64, 0), ("f32", C.F32, C.FLAG_MASS_FIX)):
        s = Solver(w["nx"], w["ny"], w["mobility"], w["width"], w["cfl"], recon=C.UPWIND5,
                   precision=prec, vel_kind=w["vel_kind"], vel_param=w["vel_param"],
                   flags=flags).init(w["phi0"])
        rows = s.tune()
        wall, ev_ms = time_steps(s, steps, warmup)
        k_ms = time_kernel_only(s, min(steps, 50))
        esize = 8 if prec == C.F64 else 4
        achieved = WORDS_PER_LU * esize * lus / (k_ms * 1e-3) / 1e9
        out[name] = {"value": round(lus * steps / (ev_ms * 1e-3) / 1e6, 1), "unit": "MLUPS",
                     "ms_per_step": round(ev_ms / steps, 4), "kernel_ms": round(k_ms, 4),
                     "achieved": round(achieved, 1), "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "tile_rows": rows, "bytes_per_lu": WORDS_PER_LU * esize}
        del s
        torch.cuda.empty_cache()
    return dict(out["f64"], dtype="f64", kernel="step_kernel, upwind-5 (wide patch)",
                fp32=dict(out["f32"], dtype="f32", mass_correction="fused, every step"))


def bench_shard_share(w, steps, warmup):
    """FP64 on one GPU's share of an 8-way row-slab split of the headline grid:
    4096 x 512 rows of the same field, periodic (a slab would take its 3 halo
    rows from its neighbours instead; the kernel's work per row is the same)."""
    import torch
    from paper_2007_07760_amd import _lib as C
    from paper_2007_07760_amd.solver import Solver
    ny = w["ny"] // 8
    s = Solver(w["nx"], ny, w["mobility"], w["width"], w["cfl"], recon=w["recon"],
               precision=C.F64, vel_kind=w["vel_kind"], vel_param=w["vel_param"]).init(
                   w["phi0"][:ny].copy())
    rows = s.tune()
    wall, ev_ms = time_steps(s, steps, warmup)
    del s
    torch.cuda.empty_cache()
    lus = w["nx"] * ny
    return {"workload": f"{w['nx']}x{ny}: one GPU's share of an 8-way row-slab split of the "
                        f"{w['nx']}x{w['ny']} grid (halo exchange not included)",
            "value": round(lus * steps / (ev_ms * 1e-3) / 1e6, 1), "unit": "MLUPS",
            "ms_per_step": round(ev_ms / steps, 4), "dtype": "f64", "tile_rows": rows}


def bench_batch_kernel(steps, rows):
    """The batch kernel alone on the C4 grids (for counter runs): tile height
    `rows`, `steps` plain launches (no autotuner, no graph, no one-grid path)."""
    import torch
    from paper_2007_07760_amd import _lib as C
    from paper_2007_07760_amd import inputs as I
    from paper_2007_07760_amd.batch import Batch
    from paper_2007_07760_amd.solver import Solver
    grids = I.batch_grids(256, seed=0)
    b = Batch(len(grids), C.F32, C.UPWIND3, C.FLAG_MASS_FIX)
    sol = [Solver(g["nx"], g["ny"], g["mobility"], g["width"], g["cfl"], recon=g["recon"],
                  precision=C.F32, vel_kind=g["vel_kind"], vel_param=g["vel_param"],
                  flags=C.FLAG_MASS_FIX).init(I.batch_phi0(g)) for g in grids]
    for k, s in enumerate(sol):
        b.set(k, s, s.step_index + steps)
    b.tile_rows = rows
    b.commit()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    b.step(steps, graph_steps=0)
    e1.record()
    torch.cuda.synchronize()
    cells = sum(g["nx"] * g["ny"] for g in grids)
    return {"workload": f"256 periodic grids (c4), {cells} cells, FP32 + fused mass correction",
            "tile_rows": rows, "steps": steps,
            "ms_per_step": round(e0.elapsed_time(e1) / steps, 4)}


def bench_batched(steps):
    """C4: 256 independent grids, FP32 + fused mass correction, upwind-3.
    Batched: one persistent kernel per step over all grids, hipGraph replays
    of 50 steps, tile height from the autotuner.  Plain: each grid alone, one
    step kernel (+ its mass-correction kernel) per launch."""
    import torch
    from paper_2007_07760_amd import _lib as C
    from paper_2007_07760_amd import inputs as I
    from paper_2007_07760_amd.batch import Batch
    from paper_2007_07760_amd.solver import Solver
    grids = I.batch_grids(256, seed=0)
    cells = sum(g["nx"] * g["ny"] for g in grids)

    def make():
        out = []
        for g in grids:
            out.append(Solver(g["nx"], g["ny"], g["mobility"], g["width"], g["cfl"],
                              recon=g["recon"], precision=C.F32, vel_kind=g["vel_kind"],
                              vel_param=g["vel_param"], flags=C.FLAG_MASS_FIX)
                       .init(I.batch_phi0(g)))
        return out

    sol = make()
    b = Batch(len(grids), C.F32, C.UPWIND3, C.FLAG_MASS_FIX)
    for k, s in enumerate(sol):
        b.set(k, s, steps + 10)
    b.commit()
    b.step(2, graph_steps=0)
    rows = b.tune(reps=3)
    b.step(8, graph_steps=0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    b.step(steps, graph_steps=50)
    e1.record()
    torch.cuda.synchronize()
    t_batch = e0.elapsed_time(e1) * 1e-3
    st = b.sync()
    assert all(int(x) == steps + 10 for x in st[:len(grids), 0])
    del b, sol
    sol = make()
    for s in sol:
        s.step(2)
    torch.cuda.synchronize()
    e0.record()
    for s in sol:
        s.step(steps)
    e1.record()
    torch.cuda.synchronize()
    t_plain = e0.elapsed_time(e1) * 1e-3
    del sol
    torch.cuda.empty_cache()
    lus = cells * steps
    return {"workload": f"256 periodic grids, sides log-uniform 32-512 (seed 0), {cells} "
                        f"cells in all, upwind-3, FP32 + fused mass correction, {steps} "
                        "steps each",
            "value": round(lus / t_batch / 1e6, 1), "unit": "MLUPS",
            "plain_one_grid_per_launch": round(lus / t_plain / 1e6, 1),
            "speedup": round(t_plain / t_batch, 2), "tile_rows": rows,
            "graph_steps": 50, "seconds": round(t_batch, 4),
            "plain_seconds": round(t_plain, 4)}


def bench_serving(count):
    """C5, scaled to a bench run: Poisson arrivals at 200/s of square solves,
    sides log-uniform 64-1024, 500-5000 steps, FP32; continuous batching vs
    one-at-a-time in arrival order on the same trace, then the batched server
    again at ~70 % of its measured capacity."""
    import numpy as np
    from paper_2007_07760_amd import inputs as I
    from paper_2007_07760_amd import serve as S
    trace = I.serve_trace(count=count, rate=200.0, nmin=64, nmax=1024, smin=500,
                          smax=5000, seed=0)
    srv = S.Server(slots=64, budget_bytes=48 << 30, graph_steps=16)
    sample = [r["id"] for r in trace[:: max(1, len(trace) // 8)]][:8]
    res = srv.run(trace, keep_phi=sample)
    sat = S.summary(res)
    fifo = S.summary(S.run_fifo(trace))
    same = all(np.array_equal(r.phi, S.run_alone(trace[r.id])) for r in res
               if r.phi is not None)
    lu_req = sat["lattice_updates"] / len(trace)
    rate = 0.7 * sat["mlups"] * 1e6 / lu_req
    trace2 = I.serve_trace(count=count, rate=rate, nmin=64, nmax=1024, smin=500,
                           smax=5000, seed=1)
    unsat = S.summary(srv.run(trace2))
    del srv

    def r4(d):
        return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in d.items()}
    return {"workload": f"{count} requests, Poisson 200/s, N 64-1024 log-uniform, "
                        "500-5000 steps, single vortex / rotation, upwind-3, FP32",
            "batched": r4(sat), "one_at_a_time": r4(fifo),
            "mix_equals_alone_sampled": bool(same), "samples": len(sample),
            "unsaturated": dict(r4(unsat), rate_per_s=round(rate, 1))}


def _cpu_model() -> str:
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w):
    """The FP64 oracle as it stands, on this host's cores, on bounded samples
    of the measured workloads: the first CPU_STEPS steps of the 4096^2 grid
    (the `value`, the same workload as the GPU line) and the first steps of the
    64^2, 256^2 and 512^2 cases."""
    import oracle
    from paper_2007_07760_amd import inputs as I

    def sample(wl, steps):
        p = oracle.Params(wl["nx"], wl["ny"], wl["mobility"], wl["width"], wl["cfl"],
                          wl["recon"], wl["vel_kind"], wl["vel_param"])
        s = oracle.State(p, wl["phi0"])
        t0 = time.perf_counter()
        s.run(steps)
        dt = time.perf_counter() - t0
        return wl["nx"] * wl["ny"] * steps / dt / 1e6, dt

    others = {}
    for name, steps in (("c1", 400), ("c2", 100), ("c3_512", 24)):
        wl = I.workload(name)
        v, dt = sample(wl, steps)
        others[f"{name} {wl['nx']}x{wl['ny']}, {steps} steps"] = {
            "mlups": round(v, 2), "seconds": round(dt, 2)}
    v, dt = sample(w, CPU_STEPS)
    cores = oracle.threads()
    # one core: the 256^2 case again
    oracle.set_threads(1)
    v1, dt1 = sample(I.workload("c2"), 40)
    oracle.set_threads(cores)
    return {"value": round(v, 2), "unit": "MLUPS",
            "cores": cores, "cpu": _cpu_model(), "kind": "oracle",
            "sample": f"{CPU_STEPS} steps (n=0..{CPU_STEPS - 1}) of the {w['nx']}x{w['ny']} "
                      f"workload, FP64, {dt:.1f} s",
            "other_samples": others,
            "single_thread": {"c2 256x256, 40 steps": {"mlups": round(v1, 2),
                                                       "seconds": round(dt1, 2)}}}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(2)
    from paper_2007_07760_amd import inputs as I
    from paper_2007_07760_amd import _lib as C
    from paper_2007_07760_amd.solver import Solver

    w = I.workload("h1")
    n = args.size
    if n != w["nx"]:
        w = dict(w, nx=n, ny=n, phi0=I.random_circles(n, n, 64, 20.0 * n / 4096,
                                                      200.0 * n / 4096, 4.0, 0))
    lus = w["nx"] * w["ny"]
    if args.batch_kernel_rows:
        print(json.dumps({"batch_kernel": bench_batch_kernel(args.batch_steps,
                                                             args.batch_kernel_rows)}),
              flush=True)
        return
    if args.only_batch:
        print(json.dumps({"batched": bench_batched(args.batch_steps)}), flush=True)
        return
    results = {}
    for prec_name, prec in (("f64", C.F64), ("f32", C.F32)):
        if args.only and args.only != prec_name:
            continue
        tile = args.tile_rows if prec == C.F64 else args.tile_rows_f32
        s = Solver(w["nx"], w["ny"], w["mobility"], w["width"], w["cfl"],
                   recon=w["recon"], precision=prec, vel_kind=w["vel_kind"],
                   vel_param=w["vel_param"], tile_rows=tile,
                   flags=C.FLAG_MASS_FIX if prec == C.F32 else 0).init(w["phi0"])
        # tile height: measured on this state before the warm-up (dugks_tune
        # leaves the state unchanged)
        rows, source = pick_tile(s, tile, f"traffic_h1_{prec_name}")
        wall, ev_ms = time_steps(s, args.steps, args.warmup)
        k_ms = time_kernel_only(s, min(args.steps, 50))
        esize = 8 if prec == C.F64 else 4
        alg_bytes = WORDS_PER_LU * esize * lus
        achieved = alg_bytes / (k_ms * 1e-3) / 1e9
        results[prec_name] = dict(
            wall=wall, ev_ms=ev_ms, kernel_ms=k_ms, achieved=achieved,
            mlups=lus * args.steps / (ev_ms * 1e-3) / 1e6, tile_rows=rows, tile_source=source,
            traffic=profile_traffic(prec_name, rows), step=s.step_index,
            phi=s.phi().double().cpu().numpy(), mass0=s.mass0(), mass=s.mass())
        del s
        torch.cuda.empty_cache()
        progress(f"{prec_name} {results[prec_name]['mlups']:.0f} MLUPS")
    copy_gbs = copy_bandwidth()
    head = "f64" if "f64" in results else "f32"
    r = results[head]
    line = {
        "metric": "MLUPS (DUGKS D2Q9 step, FP64 and FP32) and % HBM roofline",
        "value": round(r["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ev_ms"] / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head,
        "data": "synthetic",
        "config": {"workload": f"h1: {w['nx']}x{w['ny']} periodic D2Q9 DUGKS T2 step, "
                               "upwind-3 isotropic reconstruction, W=4, M=0.01, C=0.5, "
                               "64 tanh circles in rigid rotation",
                   "nx": w["nx"], "ny": w["ny"], "recon": "upwind3",
                   "tile_rows": r["tile_rows"], "tile_source": r["tile_source"]},
        "roofline": {"bound": "hbm", "achieved": round(r["achieved"], 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(r["achieved"] / HBM_PEAK_GBS, 4),
                     "target_frac": TARGET_FRAC,
                     "target_met": r["achieved"] / HBM_PEAK_GBS >= TARGET_FRAC,
                     "traffic": r["traffic"],
                     "kernel": "step_kernel (fused reconstruction + flux + update)",
                     "kernel_ms": round(r["kernel_ms"], 4),
                     "bytes_per_lu": WORDS_PER_LU * (8 if head == "f64" else 4)},
        "copy_bandwidth_gbs": round(copy_gbs, 1),
        "clock_warmup_steps": CLOCK_WARMUP_STEPS,
    }
    if "f32" in results and head != "f32":
        f = results["f32"]
        import numpy as np
        d = results["f32"]["phi"] - r["phi"]
        acc = {"step": f["step"],
               "l2": float(f"{np.sqrt((d * d).sum() / (r['phi'] ** 2).sum()):.3g}"),
               "linf": float(f"{np.abs(d).max():.3g}"),
               "relative_mass_drift": float(f"{abs(f['mass'] - f['mass0']) / f['mass0']:.3g}")}
        acc["target_met"] = (acc["l2"] <= TARGET_FP32_L2
                             and acc["relative_mass_drift"] <= TARGET_FP32_DRIFT)
        assert f["step"] == r["step"]
        line["fp32"] = {"value": round(f["mlups"], 1), "unit": "MLUPS",
                        "vs_fp64": acc,
                        "ms_per_step": round(f["ev_ms"] / args.steps, 4),
                        "mass_correction": "fused, every step",
                        "kernel_ms": round(f["kernel_ms"], 4),
                        "achieved": round(f["achieved"], 1),
                        "frac": round(f["achieved"] / HBM_PEAK_GBS, 4),
                        "traffic": f["traffic"], "bytes_per_lu": WORDS_PER_LU * 4,
                        "tile_rows": f["tile_rows"], "tile_source": f["tile_source"]}
    if not args.no_t3s3 and not args.only:
        line["t3s3"] = bench_t3s3(w, args.steps, args.warmup, args.tile_rows_t3s3)
        progress("t3s3 done")
    if not args.no_t2s5 and not args.only:
        line["t2s5"] = bench_t2s5(w, args.steps, args.warmup)
        progress("t2s5 done")
    if not args.no_shard and not args.only:
        line["shard_share"] = bench_shard_share(w, args.steps, args.warmup)
        progress("shard_share done")
    if not args.no_batch and not args.only:
        line["batched"] = bench_batched(args.batch_steps)
        progress("batched done")
    if not args.no_serve and not args.only:
        line["serving"] = bench_serving(args.serve_requests)
        progress("serving done")
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w)
        progress("cpu_baseline done")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
