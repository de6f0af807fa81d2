"""Continuous-batching service of interface-tracking solves on one GPU.

Requests (grid size, step count, velocity field, initial circle) arrive over
time.  The server admits each one as soon as a batch slot is free and its
state fits in the HBM budget (a first-fit pool over one device buffer), draws
its phi0 in device memory, and attaches it to one batch (include/dugks.h:
one persistent kernel per step over every active grid, K-step hipGraph
replays).  Grids leave the batch when they reach their own step count; their
phi is copied to pinned host memory and the request completes when the copy
has landed.  A grid whose state turns non-finite (the library's status
DUGKS_ENUMERIC, from its first state or its per-step mass sum) is stopped by
the batch and its request fails alone, with that status and no result.  Requests that arrive while others are on the GPU join before
the next group of K steps.  The baseline runs the same requests one at a time, in arrival
order, each with its own per-step launches (dugks_step).

Host-side scheduling only: every step of every solve runs in libdugks.so.
"""
from __future__ import annotations

import argparse
import collections
import dataclasses
import json
import sys
import time

import numpy as np
import torch

from . import _lib as C
from . import inputs as I
from .batch import Batch
from .solver import Solver

ALIGN = 256


class Pool:
    """First-fit allocator over one device buffer of `nbytes` (the HBM budget
    for request states).  Offsets are 256-byte aligned."""

    def __init__(self, nbytes: int, device):
        self.nbytes = int(nbytes) // ALIGN * ALIGN
        self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        self.base = self.buf.data_ptr()
        self.pad = (-self.base) % ALIGN
        self.free = [(self.pad, self.nbytes - self.pad)]   # (offset, size), sorted
        self.used = 0
        self.peak = 0

    def alloc(self, n: int):
        n = (int(n) + ALIGN - 1) // ALIGN * ALIGN
        for k, (off, size) in enumerate(self.free):
            if size >= n:
                if size == n:
                    self.free.pop(k)
                else:
                    self.free[k] = (off + n, size - n)
                self.used += n
                self.peak = max(self.peak, self.used)
                return off
        return None

    def release(self, off: int, n: int) -> None:
        n = (int(n) + ALIGN - 1) // ALIGN * ALIGN
        self.used -= n
        self.free.append((off, n))
        self.free.sort()
        merged = []
        for o, s in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + s)
            else:
                merged.append((o, s))
        self.free = merged

    def view(self, off: int, n: int) -> torch.Tensor:
        return self.buf[off:off + n]


def make_solver(req: dict, device, state=None) -> Solver:
    return Solver(req["nx"], req["ny"], req["mobility"], req["width"], req["cfl"],
                  recon=req["recon"], precision=C.F32, vel_kind=req["vel_kind"],
                  vel_param=req["vel_param"], flags=C.FLAG_MASS_FIX, device=device,
                  state=state)


def request_phi0(req: dict, device) -> torch.Tensor:
    cx, cy, r, periodic = req["circle"]
    return I.tanh_circle_torch(req["nx"], req["ny"], cx, cy, r, req["width"], periodic,
                               device)


def state_bytes(req: dict) -> int:
    p = C.make_params(req["nx"], req["ny"], req["mobility"], req["width"], req["cfl"],
                      req["recon"], C.F32, req["vel_kind"], req["vel_param"],
                      C.FLAG_MASS_FIX)
    plan = C.dugks_plan_create(p)
    try:
        return C.dugks_state_bytes(plan)
    finally:
        C.dugks_plan_destroy(plan)


@dataclasses.dataclass
class Job:
    req: dict
    solver: Solver
    off: int
    nbytes: int
    admitted: float
    first_round: int      # the first batch round the job takes part in


@dataclasses.dataclass
class Result:
    id: int
    arrival: float
    admitted: float
    done: float
    cells: int
    steps: int
    phi: np.ndarray | None
    status: int = C.OK       # C.ENUMERIC: the solve blew up; no result

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def _wait_until(t0: float, t: float) -> None:
    while True:
        d = t - (time.perf_counter() - t0)
        if d <= 0:
            return
        time.sleep(min(d, 2e-4))


class Server:
    """Continuous batching over `slots` batch slots and a `budget_bytes` pool."""

    def __init__(self, slots: int = 64, budget_bytes: int = 16 << 30, graph_steps: int = 16,
                 tile_rows: int | None = None, device="cuda"):
        self.device = torch.device(device)
        self.slots = int(slots)
        self.K = int(graph_steps)
        self.batch = Batch(self.slots, C.F32, C.UPWIND3, C.FLAG_MASS_FIX, device=self.device)
        if tile_rows:
            self.batch.tile_rows = tile_rows
        self.pool = Pool(budget_bytes, self.device)
        self._ctr = [torch.zeros(2 * self.slots, dtype=torch.int64, pin_memory=True)
                     for _ in range(2)]
        self._stat = [torch.zeros(self.slots, dtype=torch.int32, pin_memory=True)
                      for _ in range(2)]
        self._ev = [torch.cuda.Event(), torch.cuda.Event()]

    def run(self, trace: list, keep_phi=(), progress=None) -> list[Result]:
        """Serve `trace` (requests with arrival times in seconds from the
        start); returns one Result per request, in id order.  phi is kept on
        the host for the ids in `keep_phi`; `progress(done, total)` is called
        about every 30 s."""
        keep = set(keep_phi)
        t_note = time.perf_counter()
        dev = self.device
        self.budget_blocked_rounds = 0
        self.slots_peak = 0
        too_big = [r["id"] for r in trace if state_bytes(r) > self.pool.nbytes - ALIGN]
        if too_big:
            raise ValueError(f"requests {too_big[:5]} do not fit in the HBM budget")
        pending = collections.deque(sorted(trace, key=lambda r: r["arrival"]))
        queue: list[dict] = []
        free = list(range(self.slots - 1, -1, -1))
        active: dict[int, Job] = {}
        finishing = []
        results: dict[int, Result] = {}
        sizes = {}
        rounds = 0
        last = None           # index of the counter buffer of the last round
        round_of = [-1, -1]   # round whose counters each buffer holds
        t0 = time.perf_counter()
        with torch.cuda.device(dev):
            while pending or queue or active or finishing:
                now = time.perf_counter() - t0
                while pending and pending[0]["arrival"] <= now:
                    queue.append(pending.popleft())
                changed = False
                # admission: arrival order, later requests may pass one that
                # does not fit yet
                k = 0
                blocked = False
                while k < len(queue) and free:
                    req = queue[k]
                    nb = sizes.get(req["id"]) or sizes.setdefault(req["id"], state_bytes(req))
                    off = self.pool.alloc(nb)
                    if off is None:
                        blocked = True
                        k += 1
                        continue
                    queue.pop(k)
                    slot = free.pop()
                    s = make_solver(req, dev, self.pool.view(off, nb))
                    s.init(request_phi0(req, dev))
                    self.batch.set(slot, s, req["steps"])
                    active[slot] = Job(req, s, off, nb, time.perf_counter() - t0, rounds)
                    changed = True
                if changed:
                    self.batch.commit()
                # rounds in which a free slot stayed empty for want of memory
                self.budget_blocked_rounds += int(blocked and bool(free))
                self.slots_peak = max(self.slots_peak, len(active))
                if active:
                    j = rounds & 1
                    self.batch.step(self.K, graph_steps=self.K)
                    self.batch.steps_async(self._ctr[j])
                    self.batch.status_async(self._stat[j])
                    self._ev[j].record()
                    round_of[j] = rounds
                    rounds += 1
                    # completions of the previous round (one round in flight)
                    if last is not None:
                        self._ev[last].synchronize()
                        ctr = self._ctr[last].numpy().reshape(self.slots, 2)
                        stat = self._stat[last].numpy()
                        for slot in [s for s, jb in active.items()
                                     if jb.first_round <= round_of[last]
                                     and (ctr[s, 0] >= jb.req["steps"] or stat[s] != C.OK)]:
                            jb = active.pop(slot)
                            if stat[slot] != C.OK:
                                # blown up: the batch has stopped it; fail it alone
                                r = jb.req
                                results[r["id"]] = Result(
                                    r["id"], r["arrival"], jb.admitted,
                                    time.perf_counter() - t0, r["nx"] * r["ny"],
                                    int(ctr[slot, 0]), None, int(stat[slot]))
                            else:
                                jb.solver.step_index = jb.req["steps"]
                                phi = jb.solver.phi()
                                host = torch.empty(phi.shape, dtype=phi.dtype,
                                                   pin_memory=True)
                                host.copy_(phi, non_blocking=True)
                                ev = torch.cuda.Event()
                                ev.record()
                                finishing.append((jb, host, ev))
                            self.batch.clear(slot)
                            free.append(slot)
                            self.pool.release(jb.off, jb.nbytes)
                            changed = True
                        if changed:
                            self.batch.commit()
                    last = j
                else:
                    last = None
                    if finishing:
                        finishing[0][2].synchronize()
                    elif pending and not queue:
                        _wait_until(t0, pending[0]["arrival"])
                still = []
                for jb, host, ev in finishing:
                    if ev.query():
                        r = jb.req
                        results[r["id"]] = Result(
                            r["id"], r["arrival"], jb.admitted, time.perf_counter() - t0,
                            r["nx"] * r["ny"], r["steps"],
                            host.numpy().copy() if r["id"] in keep else None)
                    else:
                        still.append((jb, host, ev))
                finishing = still
                if progress and time.perf_counter() - t_note > 30.0:
                    t_note = time.perf_counter()
                    progress(len(results), len(trace))
        return [results[k] for k in sorted(results)]


def run_alone(req: dict, device="cuda") -> np.ndarray:
    """One request on its own: plain per-step launches; phi on the host."""
    s = make_solver(req, torch.device(device))
    s.init(request_phi0(req, s.device))
    s.step(req["steps"])
    return s.phi().cpu().numpy()


def run_fifo(trace: list, keep_phi=(), device="cuda", progress=None) -> list[Result]:
    """The baseline: requests one at a time in arrival order, each with its
    own memory and per-step launches."""
    keep = set(keep_phi)
    t_note = time.perf_counter()
    dev = torch.device(device)
    out = []
    t0 = time.perf_counter()
    with torch.cuda.device(dev):
        for r in sorted(trace, key=lambda r: r["arrival"]):
            _wait_until(t0, r["arrival"])
            t_adm = time.perf_counter() - t0
            s = make_solver(r, dev)
            s.init(request_phi0(r, dev))
            s.step(r["steps"])
            phi = s.phi().cpu().numpy()      # waits for the stream
            out.append(Result(r["id"], r["arrival"], t_adm, time.perf_counter() - t0,
                              r["nx"] * r["ny"], r["steps"],
                              phi if r["id"] in keep else None))
            del s
            if progress and time.perf_counter() - t_note > 30.0:
                t_note = time.perf_counter()
                progress(len(out), len(trace))
    return sorted(out, key=lambda x: x.id)


def summary(results: list[Result]) -> dict:
    failed = sum(1 for r in results if r.status != C.OK)
    lat = np.array([r.latency for r in results])
    lus = sum(r.cells * r.steps for r in results)
    t_first = min(r.arrival for r in results)
    t_last = max(r.done for r in results)
    return dict(requests=len(results), mlups=lus / (t_last - t_first) / 1e6,
                makespan_s=t_last - t_first, p50_s=float(np.percentile(lat, 50)),
                p99_s=float(np.percentile(lat, 99)), mean_s=float(lat.mean()),
                lattice_updates=int(lus), failed=failed)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description="Serve a synthetic request stream of "
                                 "interface-tracking solves; print one JSON line.")
    ap.add_argument("--count", type=int, default=1000)
    ap.add_argument("--rate", type=float, default=200.0, help="mean arrivals per second")
    ap.add_argument("--nmin", type=int, default=64)
    ap.add_argument("--nmax", type=int, default=4096)
    ap.add_argument("--smin", type=int, default=500)
    ap.add_argument("--smax", type=int, default=20000)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--mode", choices=["batched", "fifo"], default="batched")
    ap.add_argument("--slots", type=int, default=64)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--graph-steps", type=int, default=16)
    ap.add_argument("--samples", type=int, default=16,
                    help="requests whose result is compared with an alone run")
    args = ap.parse_args(argv)
    if not torch.cuda.is_available():
        print("serving needs a HIP device", file=sys.stderr)
        return 2
    trace = I.serve_trace(args.count, args.rate, args.nmin, args.nmax, args.smin, args.smax,
                          args.seed)
    step = max(1, len(trace) // max(1, args.samples))
    sample = [r["id"] for r in trace[::step]][:args.samples]

    def note(done, total):
        print(f"progress {done}/{total}", file=sys.stderr, flush=True)

    if args.mode == "batched":
        srv = Server(args.slots, int(args.budget_gb * (1 << 30)), args.graph_steps)
        res = srv.run(trace, keep_phi=sample, progress=note)
        extra = {"pool_peak_gb": round(srv.pool.peak / (1 << 30), 3), "slots": args.slots,
                 "budget_gb": args.budget_gb, "slots_peak": srv.slots_peak,
                 "budget_blocked_rounds": srv.budget_blocked_rounds,
                 "graph_steps": args.graph_steps, "tile_rows": srv.batch.tile_rows}
        del srv
    else:
        res = run_fifo(trace, keep_phi=sample, progress=note)
        extra = {}
    same = [r.id for r in res if r.phi is not None and
            not np.array_equal(r.phi, run_alone(trace[r.id]))]
    out = dict(summary(res), mode=args.mode, count=args.count, rate=args.rate,
               sizes=[args.nmin, args.nmax], steps=[args.smin, args.smax], seed=args.seed,
               samples_checked=len(sample), samples_differing=same, **extra)
    print(json.dumps({k: (round(v, 4) if isinstance(v, float) else v)
                      for k, v in out.items()}), flush=True)
    return 0 if not same else 1


if __name__ == "__main__":
    sys.exit(main())
