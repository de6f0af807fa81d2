"""FP64 CPU oracle of the D2Q9 DUGKS step (T2 and T3S3) -- test infrastructure only.

Only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library neither imports nor
links it, and shares no code with it.

The arithmetic lives in ``dugks_oracle.c`` (plain C, FP64, built with
``-ffp-contract=off``); this module compiles it with gcc when the shared object
is missing and wraps it with ctypes for numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dugks_oracle.c")
# "plain": every expression rounded as written (-ffp-contract=off): the oracle.
# "fma": the same source with a*b+c contracted to fused multiply-adds.  It is
# not a reference for values; it is another rounding of the identical
# arithmetic, used to measure how far rounding alone moves the method (the
# normal grad(phi)/|grad(phi)| is ill-conditioned where the gradient vanishes
# and theta does not).
# "aniso": a planted mistake for one test -- the normal of Eq. (2) from two-point
# axis differences, the non-isotropic choice Sec. III.A warns against -- so that
# the run-level isotropy check can be shown to catch it.  Never a reference.
_LIBS = {"plain": os.path.join(_HERE, "libdugks_oracle.so"),
         "fma": os.path.join(_HERE, "libdugks_oracle_fma.so"),
         "aniso": os.path.join(_HERE, "libdugks_oracle_aniso.so")}
_FLAGS = {"plain": ["-ffp-contract=off"], "fma": ["-ffp-contract=fast", "-mfma"],
          "aniso": ["-ffp-contract=off", "-DORC_PLANT_ANISOTROPIC_NORMAL"]}
_LIB = _LIBS["plain"]

CENTRAL2, UPWIND3, CENTRAL4, UPWIND5 = 0, 1, 2, 3   # UPWIND5: T2S5 (oracle only)
T2, T3S3 = 0, 1
VEL_UNIFORM, VEL_ROTATION, VEL_SINGLE_VORTEX, VEL_DEFORMATION, VEL_ARRAYS = range(5)


def build(force: bool = False, variant: str = "plain") -> str:
    """Compile the oracle with gcc (OpenMP over rows) into its shared object
    (again whenever the source is newer than it)."""
    out = _LIBS[variant]
    stale = (not os.path.exists(out) or
             os.path.getmtime(out) < max(os.path.getmtime(_SRC),
                                         os.path.getmtime(os.path.join(_HERE, "dugks_oracle.h"))))
    if force or stale:
        tmp = out + ".tmp"
        cmd = ["gcc", "-O2", *_FLAGS[variant], "-fopenmp", "-std=c11",
               "-D_DEFAULT_SOURCE", "-Wall", "-Wextra", "-shared", "-fPIC",
               _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)
    return out


def build_all(force: bool = False) -> None:
    for v in _LIBS:
        build(force, v)


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("mobility", ctypes.c_double), ("width", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("recon", ctypes.c_int), ("vel_kind", ctypes.c_int),
        ("vel_param", ctypes.c_double * 6),
        ("u_arr", ctypes.c_void_p), ("v_arr", ctypes.c_void_p),
        ("dtphiu_zero", ctypes.c_int),
        ("scheme", ctypes.c_int),
    ]


_libs: dict = {}


def lib(variant: str = "plain"):
    if variant not in _libs:
        L = ctypes.CDLL(build(variant=variant))
        P = ctypes.POINTER(_Params)
        dp = ctypes.c_void_p
        L.oracle_step.argtypes = [P, ctypes.c_long, dp, dp, dp, dp]
        L.oracle_init.argtypes = [P, dp, dp, dp]
        L.oracle_run.argtypes = [P, ctypes.c_long, ctypes.c_long, dp, dp]
        L.oracle_reconstruct.argtypes = [P, dp, dp, dp]
        L.oracle_grad.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp]
        L.oracle_hess.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, dp]
        L.oracle_phi.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp]
        L.oracle_mass.argtypes = [ctypes.c_int, ctypes.c_int, dp]
        L.oracle_mass.restype = ctypes.c_double
        L.oracle_velocity.argtypes = [P, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double,
                                      ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double)]
        L.oracle_feq_source.argtypes = [ctypes.c_double] * 8 + [dp, dp]
        L.oracle_aux_shift.argtypes = [ctypes.c_double] * 6
        L.oracle_aux_shift.restype = ctypes.c_double
        L.oracle_threads.restype = ctypes.c_int
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_set_threads.restype = None
        _libs[variant] = L
    return _libs[variant]


def _ptr(a: np.ndarray) -> int:
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


@dataclass
class Params:
    """Problem statement of one grid (grid, velocity, mobility, width, CFL, scheme)."""
    nx: int
    ny: int
    mobility: float
    width: float
    cfl: float
    recon: int = UPWIND3
    vel_kind: int = VEL_UNIFORM
    vel_param: tuple = (0.0, 0.0)
    u_arr: np.ndarray | None = None
    v_arr: np.ndarray | None = None
    dtphiu_zero: bool = False
    scheme: int = 0          # T2 (0) or T3S3 (1)
    _keep: list = field(default_factory=list, repr=False)

    def c(self) -> _Params:
        p = _Params()
        p.nx, p.ny = self.nx, self.ny
        p.mobility, p.width, p.cfl = self.mobility, self.width, self.cfl
        p.recon, p.vel_kind = self.recon, self.vel_kind
        vp = list(self.vel_param) + [0.0] * (6 - len(self.vel_param))
        for k in range(6):
            p.vel_param[k] = float(vp[k])
        if self.vel_kind == VEL_ARRAYS:
            u = np.ascontiguousarray(self.u_arr, dtype=np.float64)
            v = np.ascontiguousarray(self.v_arr, dtype=np.float64)
            self._keep[:] = [u, v]
            p.u_arr, p.v_arr = u.ctypes.data, v.ctypes.data
        p.dtphiu_zero = int(self.dtphiu_zero)
        p.scheme = int(self.scheme)
        return p


class State:
    """f~ (9 planes) and the phi history plane of one grid, FP64, on the host."""

    def __init__(self, params: Params, phi0: np.ndarray, variant: str = "plain"):
        self.p = params
        self.variant = variant
        self.cp = params.c()
        ny, nx = params.ny, params.nx
        phi0 = np.ascontiguousarray(phi0, dtype=np.float64)
        assert phi0.shape == (ny, nx)
        self.tf = np.empty((9, ny, nx))
        self.phi_hist = np.empty((ny, nx))
        self.step_index = 0
        rc = lib(variant).oracle_init(ctypes.byref(self.cp), _ptr(phi0), _ptr(self.tf),
                               _ptr(self.phi_hist))
        assert rc == 0

    def run(self, nsteps: int) -> "State":
        rc = lib(self.variant).oracle_run(ctypes.byref(self.cp), self.step_index, nsteps,
                              _ptr(self.tf), _ptr(self.phi_hist))
        if rc != 0:
            raise MemoryError("oracle_run failed")
        self.step_index += nsteps
        return self

    def phi(self) -> np.ndarray:
        out = np.empty((self.p.ny, self.p.nx))
        lib().oracle_phi(self.p.nx, self.p.ny, _ptr(self.tf), _ptr(out))
        return out

    def mass(self) -> float:
        return lib().oracle_mass(self.p.nx, self.p.ny, _ptr(self.tf))


def step(params: Params, n: int, tf: np.ndarray, phi_prev: np.ndarray):
    """One step n -> n+1; returns (tf_next, phi_n)."""
    cp = params.c()
    tf = np.ascontiguousarray(tf, dtype=np.float64)
    phi_prev = np.ascontiguousarray(phi_prev, dtype=np.float64)
    out = np.empty_like(tf)
    ph = np.empty_like(phi_prev)
    rc = lib().oracle_step(ctypes.byref(cp), n, _ptr(tf), _ptr(phi_prev),
                           _ptr(out), _ptr(ph))
    assert rc == 0
    return out, ph


def reconstruct(params: Params, bfp: np.ndarray):
    """Face values fbar(x_b, t+h) on x-faces and y-faces from cell fbar+ planes."""
    cp = params.c()
    bfp = np.ascontiguousarray(bfp, dtype=np.float64)
    bx = np.empty_like(bfp)
    by = np.empty_like(bfp)
    lib().oracle_reconstruct(ctypes.byref(cp), _ptr(bfp), _ptr(bx), _ptr(by))
    return bx, by


def grad(a: np.ndarray):
    a = np.ascontiguousarray(a, dtype=np.float64)
    gx, gy = np.empty_like(a), np.empty_like(a)
    lib().oracle_grad(a.shape[1], a.shape[0], _ptr(a), _ptr(gx), _ptr(gy))
    return gx, gy


def hess(a: np.ndarray):
    a = np.ascontiguousarray(a, dtype=np.float64)
    hxx, hxy, hyy = np.empty_like(a), np.empty_like(a), np.empty_like(a)
    lib().oracle_hess(a.shape[1], a.shape[0], _ptr(a), _ptr(hxx), _ptr(hxy),
                      _ptr(hyy))
    return hxx, hxy, hyy


def feq_source(phi, ux, uy, theta, nvx, nvy, jx, jy):
    feq = np.empty(9)
    src = np.empty(9)
    lib().oracle_feq_source(phi, ux, uy, theta, nvx, nvy, jx, jy, _ptr(feq),
                            _ptr(src))
    return feq, src


def aux_shift(g, a, b, feq, src, tau) -> float:
    return lib().oracle_aux_shift(g, a, b, feq, src, tau)


def velocity(params: Params, x: float, y: float, t: float):
    cp = params.c()
    u, v = ctypes.c_double(), ctypes.c_double()
    lib().oracle_velocity(ctypes.byref(cp), x, y, t, ctypes.byref(u),
                          ctypes.byref(v))
    return u.value, v.value


def threads() -> int:
    return lib().oracle_threads()


def set_threads(n: int) -> None:
    """Threads of the oracle's loops from now on (e.g. 1 to time one core)."""
    lib().oracle_set_threads(int(n))


def e_phi(phi_t: np.ndarray, phi_0: np.ndarray) -> float:
    """Relative L2 error of Eq. (41)."""
    return float(np.sqrt(np.sum((phi_t - phi_0) ** 2) / np.sum(phi_0 ** 2)))
