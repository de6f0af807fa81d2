"""Host-side checks that need no GPU: the C-ABI library loads and exports
every function include/dugks.h declares; plan validation (a host-only call)
accepts and rejects what the header says; entry points reject bad arguments
before touching the device; the serving pool allocator and the seeded input
generators behave as documented."""
import math
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2007_07760_amd import _lib as C
from paper_2007_07760_amd import inputs as I


@pytest.fixture(scope="module")
def lib():
    return C.load()


def test_library_exports_every_header_function(lib):
    names = C.header_functions()
    assert len(names) >= 22
    out = subprocess.run(["nm", "-D", "--defined-only", C.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if ln.strip()}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert hasattr(lib, n)


def _p(**kw):
    base = dict(nx=64, ny=48, mobility=0.01, width=4.0, cfl=0.5, recon=C.UPWIND3,
                precision=C.F64, vel_kind=C.VEL_UNIFORM, vel_param=(0.01, 0.02))
    base.update(kw)
    flags = base.pop("flags", 0)
    tile = base.pop("tile_rows", 0)
    scheme = base.pop("scheme", 0)
    return C.make_params(flags=flags, tile_rows=tile, scheme=scheme, **base)


@pytest.mark.parametrize("recon", [C.CENTRAL2, C.UPWIND3, C.CENTRAL4, C.UPWIND5])
@pytest.mark.parametrize("prec", [C.F64, C.F32])
def test_plan_create_valid(lib, recon, prec):
    # plan creation also checks that the stencil table folds onto its compact
    # symmetric form (EINVAL otherwise)
    assert C.dugks_plan_create_status(_p(recon=recon, precision=prec)) == C.OK
    plan = C.dugks_plan_create(_p(recon=recon, precision=prec, flags=C.FLAG_MASS_FIX))
    try:
        nb = C.dugks_state_bytes(plan)
        esize = 8 if prec == C.F64 else 4
        # at least two buffers of 10 planes
        assert nb >= 2 * 10 * 64 * 48 * esize
        assert nb % 256 == 0
    finally:
        C.dugks_plan_destroy(plan)


@pytest.mark.parametrize("bad,code", [
    (dict(nx=7), C.EINVAL), (dict(ny=4), C.EINVAL), (dict(nx=70000), C.EINVAL),
    (dict(mobility=0.0), C.EINVAL), (dict(mobility=-1.0), C.EINVAL),
    (dict(mobility=math.inf), C.EINVAL), (dict(width=0.0), C.EINVAL),
    (dict(width=math.nan), C.EINVAL), (dict(cfl=0.0), C.EINVAL), (dict(cfl=1.01), C.EINVAL),
    (dict(recon=4), C.EINVAL), (dict(precision=2), C.EINVAL), (dict(vel_kind=5), C.EINVAL),
    (dict(vel_param=(math.nan, 0.0)), C.EINVAL), (dict(flags=4), C.EINVAL),
    (dict(tile_rows=-1), C.EINVAL),
    (dict(vel_kind=C.VEL_SINGLE_VORTEX, vel_param=(0.05, 0.0)), C.EINVAL),
])
def test_plan_create_rejects(lib, bad, code):
    assert C.dugks_plan_create_status(_p(**bad)) == code


def test_upwind5_only_where_provided(lib):
    """The fifth-order reconstruction: T2 plans of the analytic kinds; the
    T3S3 time scheme, velocity arrays and batches refuse it as unsupported."""
    assert C.dugks_plan_create_status(_p(recon=C.UPWIND5)) == C.OK
    assert C.dugks_plan_create_status(
        _p(recon=C.UPWIND5, scheme=C.T3S3, mobility=0.05)) == C.EUNSUPPORTED
    assert C.dugks_plan_create_status(
        _p(recon=C.UPWIND5, vel_kind=C.VEL_ARRAYS)) == C.EUNSUPPORTED
    out = __import__("ctypes").c_void_p()
    assert lib.dugks_batch_create(4, 0, C.UPWIND5, 0,
                                  __import__("ctypes").byref(out)) == C.EUNSUPPORTED


def test_velocity_arrays_plan(lib):
    """Caller-supplied velocities: the plan is valid, its state holds the two
    planes on top of the analytic kind's, and dugks_init refuses it without
    them (before touching the device)."""
    plain = C.dugks_plan_create(_p(nx=64, ny=48))
    arr = C.dugks_plan_create(_p(nx=64, ny=48, vel_kind=C.VEL_ARRAYS))
    try:
        extra = C.dugks_state_bytes(arr) - C.dugks_state_bytes(plain)
        assert 2 * 64 * 48 * 8 <= extra < 2 * 64 * 48 * 8 + 512
        assert lib.dugks_init(arr, 4096, 4096, None, None) == C.EINVAL
    finally:
        C.dugks_plan_destroy(plain)
        C.dugks_plan_destroy(arr)


def test_plan_create_edge_values(lib):
    assert C.dugks_plan_create_status(_p(cfl=1.0)) == C.OK
    assert C.dugks_plan_create_status(_p(width=math.inf)) == C.OK   # theta off
    assert C.dugks_plan_create_status(_p(nx=8, ny=8)) == C.OK
    assert C.dugks_plan_create_status(None) == C.EINVAL


def test_calls_reject_null_before_the_device(lib):
    plan = C.dugks_plan_create(_p())
    try:
        assert lib.dugks_init(None, None, None, None, None) == C.EINVAL
        assert lib.dugks_init(plan, None, None, None, None) == C.EINVAL
        assert lib.dugks_init(plan, 256 * 1000 + 8, 4096, None, None) == C.EINVAL  # misaligned
        assert lib.dugks_history(plan, None, 0, 4096, None) == C.EINVAL
        assert lib.dugks_history(plan, 4096, -1, 4096, None) == C.EINVAL
        assert lib.dugks_state_status(plan, 4096, None, None) == C.EINVAL
        assert lib.dugks_state_status(None, 4096, 4096, None) == C.EINVAL
        assert lib.dugks_batch_status(None, 4096, None) == C.EINVAL
        assert lib.dugks_step(plan, None, 0, 1, None) == C.EINVAL
        assert lib.dugks_step(plan, 4096, -1, 1, None) == C.EINVAL
        assert lib.dugks_step(plan, 4096, 0, -1, None) == C.EINVAL
        assert lib.dugks_phi(plan, None, 0, 4096, None) == C.EINVAL
        assert lib.dugks_distributions(plan, 4096, 0, None, None) == C.EINVAL
        assert lib.dugks_mass(plan, 4096, 0, None, None) == C.EINVAL
        assert lib.dugks_mass_correct(plan, None, 0, None) == C.EINVAL
        assert lib.dugks_mass0(plan, None, 4096, None) == C.EINVAL
        assert lib.dugks_batch_set(None, 0, plan, 4096, 0, 1) == C.EINVAL
        assert lib.dugks_batch_step(None, 1, 0, None) == C.EINVAL
        assert lib.dugks_batch_commit(None, None) == C.EINVAL
        assert lib.dugks_batch_tile_rows(None) == -1
        rows = __import__("ctypes").c_int32()
        prm = _p()
        by = __import__("ctypes").byref
        assert lib.dugks_tune(None, 4096, 0, 1, by(rows), None) == C.EINVAL
        assert lib.dugks_tune(by(prm), None, 0, 1, by(rows), None) == C.EINVAL
        assert lib.dugks_tune(by(prm), 4096 + 8, 0, 1, by(rows), None) == C.EINVAL
        assert lib.dugks_tune(by(prm), 4096, -1, 1, by(rows), None) == C.EINVAL
        assert lib.dugks_tune(by(prm), 4096, 0, 0, by(rows), None) == C.EINVAL
        assert lib.dugks_tune(by(prm), 4096, 0, 1, None, None) == C.EINVAL
        assert lib.dugks_tune(by(_p(cfl=2.0)), 4096, 0, 1, by(rows), None) == C.EINVAL
        out = __import__("ctypes").c_void_p()
        assert lib.dugks_batch_create(0, 0, 0, 0, __import__("ctypes").byref(out)) == C.EINVAL
        assert lib.dugks_batch_create(4, 0, 0, 8, __import__("ctypes").byref(out)) == C.EINVAL
    finally:
        C.dugks_plan_destroy(plan)


def test_strerror_and_version(lib):
    texts = {C.dugks_strerror(k) for k in range(6)}
    assert len(texts) == 6 and "ok" in texts
    assert "unknown" in C.dugks_strerror(99)
    assert C.dugks_version().startswith("dugks-gfx950")


# ------------------------------------------------------- serving host logic
def test_pool_first_fit_alignment_and_coalescing():
    import torch
    from paper_2007_07760_amd.serve import Pool
    p = Pool(10000, "cpu")
    offs = [p.alloc(n) for n in (1000, 3000, 2000)]
    assert all(o is not None and (p.base + o) % 256 == 0 for o in offs)
    assert p.alloc(10000) is None
    used = p.used
    p.release(offs[1], 3000)
    assert p.used == used - 3072
    # the freed middle block is reused first fit
    again = p.alloc(2900)
    assert again == offs[1]
    p.release(again, 2900)
    p.release(offs[0], 1000)
    p.release(offs[2], 2000)
    assert p.used == 0 and len(p.free) == 1
    assert p.peak <= p.nbytes
    assert isinstance(p.view(offs[0], 100), torch.Tensor)


def test_serve_trace_statistics():
    t = I.serve_trace(count=4000, rate=200.0, seed=5)
    gaps = np.diff([0.0] + [r["arrival"] for r in t])
    assert abs(gaps.mean() * 200.0 - 1.0) < 0.05          # Poisson mean gap 1/rate
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.08     # exponential: CV = 1
    ns = np.array([r["nx"] for r in t])
    assert ns.min() >= 64 and ns.max() <= 4096
    # log-uniform: log N has mean (ln 64 + ln 4096) / 2
    assert abs(np.log(ns).mean() - 0.5 * (math.log(64) + math.log(4096))) < 0.1
    st = np.array([r["steps"] for r in t])
    assert st.min() >= 500 and st.max() <= 20000
    kinds = {r["vel_kind"] for r in t}
    assert kinds == {I.VEL_SINGLE_VORTEX, I.VEL_ROTATION}
    for r in t[:50]:
        if r["vel_kind"] == I.VEL_ROTATION:
            corner = r["vel_param"][0] * math.hypot(r["nx"] / 2, r["ny"] / 2)
            assert corner == pytest.approx(0.05)
        else:   # the flow reverses at half the request's time
            assert r["vel_param"][1] == pytest.approx(r["steps"] * r["cfl"])
    assert I.serve_trace(count=20, seed=5) == t[:20]


def test_batch_grids_statistics():
    g = I.batch_grids(256, seed=0)
    assert len(g) == 256 and g == I.batch_grids(256, seed=0)
    for x in g:
        assert 32 <= x["nx"] <= 512 and 32 <= x["ny"] <= 512
        assert 1 <= x["circles"] <= 4
        m = min(x["nx"], x["ny"])
        assert x["rmin"] == pytest.approx(0.05 * m) and x["rmax"] == pytest.approx(0.25 * m)
        if x["vel_kind"] == I.VEL_UNIFORM:
            assert math.hypot(*x["vel_param"][:2]) <= 0.05
        else:
            assert x["vel_param"][0] * math.hypot(x["nx"] / 2, x["ny"] / 2) <= 0.05 + 1e-15
    kinds = [x["vel_kind"] for x in g]
    assert 80 < kinds.count(I.VEL_UNIFORM) < 176
    phi = I.batch_phi0(g[0])
    assert phi.shape == (g[0]["ny"], g[0]["nx"]) and 0.0 <= phi.min() and phi.max() <= 1.0


@pytest.mark.parametrize("periodic", [True, False])
def test_device_circle_matches_host_circle(periodic):
    import torch
    a = I.tanh_circle_torch(70, 50, 20.3, 31.7, 11.0, 4.0, periodic, "cpu").numpy()
    b = I.tanh_circle(70, 50, 20.3, 31.7, 11.0, 4.0, periodic=periodic)
    assert np.max(np.abs(a - b)) < 1e-14


def test_plan_t3s3_validation(lib):
    # dt < 12 tau: M = 0.02 -> tau = 0.06, 12 tau = 0.72
    assert C.dugks_plan_create_status(_p(mobility=0.02, cfl=0.5, scheme=1)) == C.OK
    assert C.dugks_plan_create_status(_p(mobility=0.02, cfl=0.73, scheme=1)) == C.EINVAL
    assert C.dugks_plan_create_status(_p(mobility=0.01, cfl=0.5, scheme=1)) == C.EINVAL
    assert C.dugks_plan_create_status(_p(mobility=0.02, cfl=0.5, scheme=2)) == C.EINVAL
    assert C.dugks_plan_create_status(_p(mobility=0.02, cfl=0.5, scheme=1,
                                         flags=C.FLAG_MASS_FIX)) == C.OK
    a = C.dugks_plan_create(_p(mobility=0.02, cfl=0.5))
    b = C.dugks_plan_create(_p(mobility=0.02, cfl=0.5, scheme=1))
    try:
        # T3S3 keeps two more buffers (f~ at t + dt/3 and Q) in its state
        assert C.dugks_state_bytes(b) > C.dugks_state_bytes(a) + 1.9 * 10 * 64 * 48 * 8
    finally:
        C.dugks_plan_destroy(a)
        C.dugks_plan_destroy(b)


def test_bench_refuses_several_gpus():
    """The benchmark measures one GPU; asked for more it exits with a message
    before touching a device."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], cwd=root,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
