"""dugks_step_many_noalloc: the batch step of many grids with its descriptors,
counters and work list in a fixed device array of the library (no device
allocation), against the batch entry point dugks_batch_step on the same grids.
Both run the same kernels on the same tiles, so the results must agree
bitwise.  Two calls in a row, the second with fewer and smaller grids: the
array keeps the first call's contents, which the second must not see."""
import ctypes

import numpy as np
import pytest

from paper_2007_07760_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2007_07760_amd import _lib
    _lib.load()
    return _lib


def _grids(lib, specs, precision, flags, scheme=0):
    from paper_2007_07760_amd.solver import Solver
    out = []
    # T3S3 needs dt < 12 tau = 36 M
    mobility = 0.02 if scheme else 0.01
    for k, (nx, ny, kind, prm) in enumerate(specs):
        r = min(nx, ny)
        phi0 = I.random_circles(nx, ny, 1 + k % 3, 0.1 * r, 0.3 * r, 4.0, seed=50 + k)
        out.append(Solver(nx, ny, mobility, 4.0, 0.5, recon=lib.UPWIND3, precision=precision,
                          vel_kind=kind, vel_param=prm, flags=flags,
                          scheme=scheme).init(phi0))
    return out


def _noalloc(lib, solvers, nsteps):
    import torch
    lib.dugks_step_many_noalloc([s.plan for s in solvers],
                                [s.state.data_ptr() for s in solvers],
                                [s.step_index for s in solvers], nsteps,
                                torch.cuda.current_stream().cuda_stream)
    for s in solvers:
        s.step_index += nsteps


def _batched(lib, solvers, nsteps, precision, flags, scheme=0):
    from paper_2007_07760_amd.batch import Batch
    b = Batch(len(solvers), precision, lib.UPWIND3, flags | (lib.BATCH_T3S3 if scheme else 0))
    for k, s in enumerate(solvers):
        b.set(k, s, s.step_index + nsteps)
    b.commit()
    b.step(nsteps, graph_steps=0)
    b.sync()


FIRST = [(130, 96, 1, (0.0008, 65.0, 48.0)), (64, 200, 2, (0.05, 900.0)),
         (37, 29, 0, (-0.04, 0.01)), (256, 48, 3, (0.03, 700.0)), (9, 8, 0, (0.02, 0.02))]
SECOND = [(40, 24, 0, (0.03, -0.02)), (20, 33, 1, (0.001, 10.0, 16.0))]


@pytest.mark.parametrize("precision,flags,scheme", [(1, 2, 0), (0, 0, 0), (0, 0, 1), (1, 2, 1)])
def test_noalloc_equals_batch_two_calls(lib, precision, flags, scheme):
    import torch
    print(f"case noalloc prec={precision} flags={flags} scheme={scheme}", flush=True)
    for specs, nsteps in ((FIRST, 17), (SECOND, 6)):
        a = _grids(lib, specs, precision, flags, scheme)
        b = _grids(lib, specs, precision, flags, scheme)
        _noalloc(lib, a, nsteps)
        _batched(lib, b, nsteps, precision, flags, scheme)
        for k in range(len(specs)):
            assert a[k].step_index == b[k].step_index == nsteps
            assert torch.equal(a[k].distributions(), b[k].distributions()), (specs[k], k)
            assert torch.equal(a[k].history(), b[k].history()), (specs[k], k)
            assert a[k].status() == lib.OK


def test_noalloc_rejects_beyond_its_limits(lib):
    import torch
    from paper_2007_07760_amd.solver import Solver
    s = Solver(64, 64, 0.01, 4.0, 0.5, recon=lib.UPWIND3).init(np.full((64, 64), 0.5))
    L = lib.load()
    st = torch.cuda.current_stream().cuda_stream
    n = 257
    plans = (ctypes.c_void_p * n)(*([s.plan] * n))
    states = (ctypes.c_void_p * n)(*([s.state.data_ptr()] * n))
    steps = (ctypes.c_int64 * n)(*([0] * n))
    assert L.dugks_step_many_noalloc(plans, states, steps, n, 1, st) == lib.EINVAL
    assert L.dugks_step_many_noalloc(plans, states, steps, 0, 1, st) == lib.EINVAL
    assert L.dugks_step_many_noalloc(plans, states, steps, 1, -1, st) == lib.EINVAL
    # a grid of 65536 x 8192 in 16-row tiles: 1130 strips x 512 segments, more
    # work items than the array holds; refused before anything is launched
    # (the state address is never used)
    prm = lib.make_params(65536, 8192, 0.01, 4.0, 0.5, lib.UPWIND3, tile_rows=16)
    plan = lib.dugks_plan_create(prm)
    try:
        one_p = (ctypes.c_void_p * 1)(plan)
        one_s = (ctypes.c_void_p * 1)(1 << 20)
        one_n = (ctypes.c_int64 * 1)(0)
        assert L.dugks_step_many_noalloc(one_p, one_s, one_n, 1, 1, st) == lib.EINVAL
    finally:
        lib.dugks_plan_destroy(plan)
