"""One grid advanced by the HIP library, with torch providing device memory and
streams.  Every step of the scheme runs in libdugks.so; this class only
allocates the state, keeps the step counter and marshals pointers."""
from __future__ import annotations

import math

import numpy as np
import torch

from . import _lib as C


class Solver:
    """A D2Q9 DUGKS solve of the conservative Allen-Cahn equation on one
    periodic nx x ny grid (see include/dugks.h for the parameters)."""

    def __init__(self, nx, ny, mobility, width, cfl, recon=C.UPWIND3,
                 precision=C.F64, vel_kind=C.VEL_UNIFORM, vel_param=(0.0, 0.0),
                 flags=0, tile_rows=0, device="cuda", state=None, scheme=0):
        if not torch.cuda.is_available():
            raise RuntimeError("Solver needs a HIP device (no CPU path exists)")
        self.params = C.make_params(nx, ny, mobility, width, cfl, recon, precision,
                                    vel_kind, vel_param, flags, tile_rows, scheme)
        self.nx, self.ny = int(nx), int(ny)
        self.precision = int(precision)
        self.dtype = torch.float64 if precision == C.F64 else torch.float32
        self.plan = C.dugks_plan_create(self.params)
        self.device = torch.device(device)
        nbytes = C.dugks_state_bytes(self.plan)
        if state is None:
            state = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        elif state.numel() < nbytes or state.data_ptr() % 256:
            raise ValueError("state memory too small or not 256-byte aligned")
        self.state = state          # uint8 device tensor (possibly a view of a pool)
        self.step_index = 0
        self._scalar = torch.empty(1, dtype=torch.float64, device=self.device)

    def __del__(self):
        plan = getattr(self, "plan", None)
        if plan and C is not None and C.dugks_plan_destroy is not None:
            C.dugks_plan_destroy(plan)
            self.plan = None

    @staticmethod
    def stream() -> int:
        return torch.cuda.current_stream().cuda_stream

    @staticmethod
    def _device_f64(a, device) -> torch.Tensor:
        a = torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)
                            if isinstance(a, np.ndarray) else a)
        return a.to(device=device, dtype=torch.float64).contiguous()

    def init(self, phi0, uv=None) -> "Solver":
        """First state from phi0 ([ny][nx]); `uv` ([2][ny][nx]: u, then v, at
        the cell centres) for plans with caller-supplied velocities."""
        phi0 = self._device_f64(phi0, self.device)
        assert tuple(phi0.shape) == (self.ny, self.nx)
        uvp = None
        if uv is not None:
            uv = self._device_f64(uv, self.device)
            assert tuple(uv.shape) == (2, self.ny, self.nx)
            uvp = uv.data_ptr()
        C.dugks_init(self.plan, self.state.data_ptr(), phi0.data_ptr(), uvp, self.stream())
        self.step_index = 0
        return self

    def step(self, nsteps: int = 1) -> "Solver":
        C.dugks_step(self.plan, self.state.data_ptr(), self.step_index, nsteps,
                     self.stream())
        self.step_index += nsteps
        return self

    def retile(self, rows: int) -> "Solver":
        """Rebuild the plan with another tile height (the state layout does not
        depend on it, and results do not either)."""
        if rows != self.params.tile_rows:
            self.params.tile_rows = int(rows)
            plan = C.dugks_plan_create(self.params)
            torch.cuda.current_stream().synchronize()   # init's staged copy has run
            C.dugks_plan_destroy(self.plan)
            self.plan = plan
        return self

    def tune(self, reps: int = 5) -> int:
        """Time the step's kernels on this state for a range of tile heights
        (dugks_tune, which leaves the state unchanged) and rebuild the plan
        with the fastest; returns the height."""
        rows = C.dugks_tune(self.params, self.state.data_ptr(), self.step_index, reps,
                            self.stream())
        self.retile(rows)
        return rows

    def phi(self) -> torch.Tensor:
        out = torch.empty((self.ny, self.nx), dtype=self.dtype, device=self.device)
        C.dugks_phi(self.plan, self.state.data_ptr(), self.step_index, out.data_ptr(),
                    self.stream())
        return out

    def distributions(self) -> torch.Tensor:
        out = torch.empty((9, self.ny, self.nx), dtype=self.dtype, device=self.device)
        C.dugks_distributions(self.plan, self.state.data_ptr(), self.step_index,
                              out.data_ptr(), self.stream())
        return out

    def history(self) -> torch.Tensor:
        """The stored phi of the previous step (the history plane)."""
        out = torch.empty((self.ny, self.nx), dtype=self.dtype, device=self.device)
        C.dugks_history(self.plan, self.state.data_ptr(), self.step_index, out.data_ptr(),
                        self.stream())
        return out

    def status(self) -> int:
        """The state's sticky status (OK, or ENUMERIC after a non-finite total);
        waits for the stream."""
        st = torch.empty(1, dtype=torch.int32, device=self.device)
        C.dugks_state_status(self.plan, self.state.data_ptr(), st.data_ptr(), self.stream())
        return int(st.item())

    def mass(self) -> float:
        C.dugks_mass(self.plan, self.state.data_ptr(), self.step_index,
                     self._scalar.data_ptr(), self.stream())
        m = float(self._scalar.item())
        if not math.isfinite(m):
            raise C.DugksError(C.ENUMERIC, "Solver.mass")
        return m

    def mass0(self) -> float:
        C.dugks_mass0(self.plan, self.state.data_ptr(), self._scalar.data_ptr(),
                      self.stream())
        return float(self._scalar.item())

    def mass_correct(self) -> "Solver":
        C.dugks_mass_correct(self.plan, self.state.data_ptr(), self.step_index,
                             self.stream())
        return self
