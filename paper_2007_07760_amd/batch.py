"""Many grids advanced by one persistent kernel (the batch calls of
include/dugks.h).  Each slot holds a Solver's plan and state; the step
counters live on the device while a state is attached, and `sync()` copies
them back into the solvers.  Argument marshalling only: every step runs in
libdugks.so."""
from __future__ import annotations

import numpy as np
import torch

from . import _lib as C
from .solver import Solver


class Batch:
    def __init__(self, capacity: int, precision=C.F32, recon=C.UPWIND3,
                 flags=C.FLAG_MASS_FIX, device="cuda"):
        if not torch.cuda.is_available():
            raise RuntimeError("Batch needs a HIP device (no CPU path exists)")
        self.capacity = int(capacity)
        self.precision, self.recon, self.flags = int(precision), int(recon), int(flags)
        self.device = torch.device(device)
        with torch.cuda.device(self.device):
            self.handle = C.dugks_batch_create(self.capacity, self.precision, self.recon,
                                               self.flags)
        self.solvers: list[Solver | None] = [None] * self.capacity
        self._steps = torch.zeros(2 * self.capacity, dtype=torch.int64, pin_memory=True)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            C.dugks_batch_destroy(h)
            self.handle = None

    @staticmethod
    def stream() -> int:
        return torch.cuda.current_stream().cuda_stream

    def set(self, slot: int, solver: Solver, target: int) -> None:
        """Attach `solver` (at its current step) to `slot` until `target`."""
        C.dugks_batch_set(self.handle, slot, solver.plan, solver.state.data_ptr(),
                          solver.step_index, int(target))
        self.solvers[slot] = solver

    def clear(self, slot: int) -> None:
        C.dugks_batch_clear(self.handle, slot)
        self.solvers[slot] = None

    def commit(self) -> None:
        C.dugks_batch_commit(self.handle, self.stream())

    def step(self, nsteps: int, graph_steps: int = 16) -> None:
        C.dugks_batch_step(self.handle, int(nsteps), int(graph_steps), self.stream())

    def status_async(self, out: torch.Tensor) -> None:
        """Queue a copy of each slot's status (int32; OK or ENUMERIC) into `out`."""
        C.dugks_batch_status(self.handle, out.data_ptr(), self.stream())

    def status(self) -> np.ndarray:
        """Status per slot, shape (capacity,); waits for the stream."""
        out = torch.zeros(self.capacity, dtype=torch.int32, pin_memory=True)
        self.status_async(out)
        torch.cuda.current_stream().synchronize()
        return out.numpy().copy()

    def steps_async(self, out: torch.Tensor) -> None:
        """Queue a copy of the (step, target) pairs into `out` (pinned int64)."""
        C.dugks_batch_steps(self.handle, out.data_ptr(), self.stream())

    def steps(self) -> np.ndarray:
        """(step, target) per slot, shape (capacity, 2); waits for the stream."""
        self.steps_async(self._steps)
        torch.cuda.current_stream().synchronize()
        return self._steps.numpy().reshape(self.capacity, 2).copy()

    def sync(self) -> np.ndarray:
        """Copy the device step counters into the attached solvers."""
        st = self.steps()
        for k, s in enumerate(self.solvers):
            if s is not None:
                s.step_index = int(st[k, 0])
        return st

    @property
    def tile_rows(self) -> int:
        return C.dugks_batch_tile_rows(self.handle)

    @tile_rows.setter
    def tile_rows(self, rows: int) -> None:
        C.dugks_batch_set_tile_rows(self.handle, int(rows))

    def tune(self, reps: int = 3) -> int:
        """Measure the tile heights on the attached grids; keep the fastest."""
        return C.dugks_batch_tune(self.handle, int(reps), self.stream())
