"""ctypes binding of the C ABI in include/dugks.h: argument marshalling only.

Every function keeps the C name; pointers are passed as integers (device
addresses from torch tensors, hipStream_t handles from torch streams).  The
library must be built (``paper_2007_07760_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB_PATH = os.path.join(PKG, "libdugks.so")
HEADER = os.path.join(ROOT, "include", "dugks.h")

OK, EINVAL, ENOMEM, EDEVICE, ENUMERIC, EUNSUPPORTED = range(6)
F64, F32 = 0, 1
CENTRAL2, UPWIND3, CENTRAL4, UPWIND5 = 0, 1, 2, 3
VEL_UNIFORM, VEL_ROTATION, VEL_SINGLE_VORTEX, VEL_DEFORMATION, VEL_ARRAYS = range(5)
T2, T3S3 = 0, 1
FLAG_DTPHIU_ZERO = 1
FLAG_MASS_FIX = 2
BATCH_T3S3 = 4      # batch flag: the batch advances T3S3 plans


class DugksError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {dugks_strerror(code)} (status {code})")


class dugks_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("mobility", ctypes.c_double), ("width", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("recon", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("vel_kind", ctypes.c_int32), ("flags", ctypes.c_int32),
        ("vel_param", ctypes.c_double * 6),
        ("tile_rows", ctypes.c_int32), ("scheme", ctypes.c_int32),
    ]


_lib = None


def load() -> ctypes.CDLL:
    """Load libdugks.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run paper_2007_07760_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    P = ctypes.POINTER(dugks_params)
    L.dugks_plan_create.argtypes = [P, ctypes.POINTER(vp)]
    L.dugks_plan_destroy.argtypes = [vp]
    L.dugks_plan_destroy.restype = None
    L.dugks_state_bytes.argtypes = [vp]
    L.dugks_state_bytes.restype = ctypes.c_size_t
    L.dugks_init.argtypes = [vp, vp, vp, vp, vp]
    L.dugks_history.argtypes = [vp, vp, i64, vp, vp]
    L.dugks_state_status.argtypes = [vp, vp, vp, vp]
    L.dugks_batch_status.argtypes = [vp, vp, vp]
    L.dugks_step_many_noalloc.argtypes = [vp, vp, vp, i32, i64, vp]
    L.dugks_step.argtypes = [vp, vp, i64, i64, vp]
    L.dugks_phi.argtypes = [vp, vp, i64, vp, vp]
    L.dugks_mass.argtypes = [vp, vp, i64, vp, vp]
    L.dugks_distributions.argtypes = [vp, vp, i64, vp, vp]
    L.dugks_mass_correct.argtypes = [vp, vp, i64, vp]
    L.dugks_mass0.argtypes = [vp, vp, vp, vp]
    L.dugks_strerror.argtypes = [ctypes.c_int]
    L.dugks_strerror.restype = ctypes.c_char_p
    L.dugks_version.restype = ctypes.c_char_p
    L.dugks_batch_create.argtypes = [i32, i32, i32, ctypes.c_uint32, ctypes.POINTER(vp)]
    L.dugks_batch_destroy.argtypes = [vp]
    L.dugks_batch_destroy.restype = None
    L.dugks_batch_set.argtypes = [vp, i32, vp, vp, i64, i64]
    L.dugks_batch_clear.argtypes = [vp, i32]
    L.dugks_batch_commit.argtypes = [vp, vp]
    L.dugks_batch_step.argtypes = [vp, i64, i32, vp]
    L.dugks_batch_steps.argtypes = [vp, vp, vp]
    L.dugks_batch_tile_rows.argtypes = [vp]
    L.dugks_batch_set_tile_rows.argtypes = [vp, i32]
    L.dugks_batch_tune.argtypes = [vp, i32, ctypes.POINTER(i32), vp]
    L.dugks_tune.argtypes = [P, vp, i64, i32, ctypes.POINTER(i32), vp]
    for name in ("dugks_plan_create", "dugks_init", "dugks_step", "dugks_phi",
                 "dugks_distributions", "dugks_history", "dugks_state_status", "dugks_batch_status",
                 "dugks_step_many_noalloc",
                 "dugks_mass", "dugks_mass_correct", "dugks_mass0",
                 "dugks_batch_create", "dugks_batch_set", "dugks_batch_clear",
                 "dugks_batch_commit", "dugks_batch_step", "dugks_batch_steps",
                 "dugks_batch_tile_rows", "dugks_batch_set_tile_rows",
                 "dugks_batch_tune", "dugks_tune"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def header_functions() -> list[str]:
    """Names of the functions include/dugks.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dugks_[a-z0-9_]+)\s*\(", text)))


def _check(rc: int, where: str) -> None:
    if rc != OK:
        raise DugksError(rc, where)


def make_params(nx, ny, mobility, width, cfl, recon=UPWIND3, precision=F64,
                vel_kind=VEL_UNIFORM, vel_param=(0.0, 0.0), flags=0,
                tile_rows=0, scheme=0) -> dugks_params:
    p = dugks_params()
    p.nx, p.ny = int(nx), int(ny)
    p.mobility, p.width, p.cfl = float(mobility), float(width), float(cfl)
    p.recon, p.precision, p.vel_kind = int(recon), int(precision), int(vel_kind)
    p.flags = int(flags)
    vp = list(vel_param) + [0.0] * (6 - len(vel_param))
    for k in range(6):
        p.vel_param[k] = float(vp[k])
    p.tile_rows = int(tile_rows)
    p.scheme = int(scheme)
    return p


def dugks_plan_create(params: dugks_params) -> int:
    out = ctypes.c_void_p()
    _check(load().dugks_plan_create(ctypes.byref(params), ctypes.byref(out)),
           "dugks_plan_create")
    return out.value


def dugks_plan_create_status(params) -> int:
    """Status of plan creation for possibly-invalid params (no exception)."""
    out = ctypes.c_void_p()
    ptr = ctypes.byref(params) if params is not None else None
    rc = load().dugks_plan_create(ptr, ctypes.byref(out))
    if rc == OK:
        load().dugks_plan_destroy(out)
    return rc


def dugks_plan_destroy(plan: int) -> None:
    load().dugks_plan_destroy(plan)


def dugks_state_bytes(plan: int) -> int:
    return load().dugks_state_bytes(plan)


def dugks_init(plan: int, state: int, phi0_dev: int, uv_dev, stream: int) -> None:
    _check(load().dugks_init(plan, state, phi0_dev, uv_dev, stream), "dugks_init")


def dugks_step(plan: int, state: int, step: int, nsteps: int, stream: int) -> None:
    _check(load().dugks_step(plan, state, step, nsteps, stream), "dugks_step")


def dugks_phi(plan: int, state: int, step: int, out_dev: int, stream: int) -> None:
    _check(load().dugks_phi(plan, state, step, out_dev, stream), "dugks_phi")


def dugks_distributions(plan: int, state: int, step: int, out_dev: int,
                        stream: int) -> None:
    _check(load().dugks_distributions(plan, state, step, out_dev, stream),
           "dugks_distributions")


def dugks_history(plan: int, state: int, step: int, out_dev: int, stream: int) -> None:
    _check(load().dugks_history(plan, state, step, out_dev, stream), "dugks_history")


def dugks_state_status(plan: int, state: int, out: int, stream: int) -> None:
    _check(load().dugks_state_status(plan, state, out, stream), "dugks_state_status")


def dugks_batch_status(batch: int, out: int, stream: int) -> None:
    _check(load().dugks_batch_status(batch, out, stream), "dugks_batch_status")


def dugks_step_many_noalloc(plans, states, steps, nsteps: int, stream: int) -> None:
    """plans, states, steps: sequences of n entries (plan handles, state device
    addresses, current steps)."""
    n = len(plans)
    P = (ctypes.c_void_p * n)(*plans)
    S = (ctypes.c_void_p * n)(*states)
    N = (ctypes.c_int64 * n)(*steps)
    _check(load().dugks_step_many_noalloc(P, S, N, n, nsteps, stream),
           "dugks_step_many_noalloc")


def dugks_mass(plan: int, state: int, step: int, out_dev: int, stream: int) -> None:
    _check(load().dugks_mass(plan, state, step, out_dev, stream), "dugks_mass")


def dugks_mass_correct(plan: int, state: int, step: int, stream: int) -> None:
    _check(load().dugks_mass_correct(plan, state, step, stream), "dugks_mass_correct")


def dugks_mass0(plan: int, state: int, out_dev: int, stream: int) -> None:
    _check(load().dugks_mass0(plan, state, out_dev, stream), "dugks_mass0")


def dugks_batch_create(capacity: int, precision: int, recon: int, flags: int = 0) -> int:
    out = ctypes.c_void_p()
    _check(load().dugks_batch_create(capacity, precision, recon, flags, ctypes.byref(out)),
           "dugks_batch_create")
    return out.value


def dugks_batch_destroy(batch: int) -> None:
    load().dugks_batch_destroy(batch)


def dugks_batch_set(batch: int, slot: int, plan: int, state: int, step: int,
                    target: int) -> None:
    _check(load().dugks_batch_set(batch, slot, plan, state, step, target), "dugks_batch_set")


def dugks_batch_clear(batch: int, slot: int) -> None:
    _check(load().dugks_batch_clear(batch, slot), "dugks_batch_clear")


def dugks_batch_commit(batch: int, stream: int) -> None:
    _check(load().dugks_batch_commit(batch, stream), "dugks_batch_commit")


def dugks_batch_step(batch: int, nsteps: int, graph_steps: int, stream: int) -> None:
    _check(load().dugks_batch_step(batch, nsteps, graph_steps, stream), "dugks_batch_step")


def dugks_batch_steps(batch: int, out: int, stream: int) -> None:
    _check(load().dugks_batch_steps(batch, out, stream), "dugks_batch_steps")


def dugks_batch_tile_rows(batch: int) -> int:
    return load().dugks_batch_tile_rows(batch)


def dugks_batch_set_tile_rows(batch: int, rows: int) -> None:
    _check(load().dugks_batch_set_tile_rows(batch, rows), "dugks_batch_set_tile_rows")


def dugks_batch_tune(batch: int, reps: int, stream: int) -> int:
    rows = ctypes.c_int32()
    _check(load().dugks_batch_tune(batch, reps, ctypes.byref(rows), stream), "dugks_batch_tune")
    return rows.value


def dugks_tune(params, state: int, step: int, reps: int, stream: int) -> int:
    rows = ctypes.c_int32()
    _check(load().dugks_tune(ctypes.byref(params), state, step, reps, ctypes.byref(rows), stream),
           "dugks_tune")
    return rows.value


def dugks_strerror(code: int) -> str:
    return load().dugks_strerror(code).decode()


def dugks_version() -> str:
    return load().dugks_version().decode()
