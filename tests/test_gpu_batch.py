"""The batch path (persistent kernel over many grids, hipGraph replays,
autotuned tile height) against the plain one-grid-per-launch path.

The two run the same march code on the same tiles' rows, and results do not
depend on the tiling, so every grid of a batch must equal its alone run
bitwise: FP32 with the fused mass correction and FP64, uneven grid sizes,
targets that stop grids at different steps, grids attached while others run,
and after the autotuner has changed the tile height.
"""
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


# (nx, ny, velocity kind, velocity parameters)
GRIDS = [
    (40, 72, 0, (0.03, -0.02)),
    (100, 64, 1, (0.0015, 50.0, 32.0)),
    (64, 200, 2, (0.05, 900.0)),
    (130, 130, 1, (0.0008, 65.0, 65.0)),
    (37, 29, 0, (-0.04, 0.01)),
    (256, 48, 3, (0.03, 700.0)),
    (9, 8, 0, (0.02, 0.02)),
]


def _phi0(nx, ny, seed):
    r = min(nx, ny)
    return I.random_circles(nx, ny, 1 + seed % 3, 0.1 * r, 0.3 * r, 4.0, seed)


def _solver(lib, g, seed, precision, flags, recon):
    from paper_2007_07760_amd.solver import Solver
    nx, ny, kind, prm = g
    return Solver(nx, ny, 0.01, 4.0, 0.5, recon=recon, precision=precision,
                  vel_kind=kind, vel_param=prm, flags=flags).init(_phi0(nx, ny, seed))


def _alone(lib, g, seed, precision, flags, recon, steps):
    return _solver(lib, g, seed, precision, flags, recon).step(steps)


@pytest.mark.parametrize("precision,flags,recon", [
    (1, 2, 1),   # FP32, fused mass correction, upwind-3
    (0, 0, 1),   # FP64, upwind-3
    (1, 0, 2),   # FP32, central-4
])
def test_batch_equals_alone(lib, precision, flags, recon):
    import torch
    from paper_2007_07760_amd.batch import Batch
    print(f"case batch prec={precision} flags={flags} recon={recon}", flush=True)
    targets = [23, 23, 10, 17, 23, 5, 23]
    b = Batch(8, precision, recon, flags)
    sol = []
    for k, g in enumerate(GRIDS):
        s = _solver(lib, g, k, precision, flags, recon)
        b.set(k, s, targets[k])
        sol.append(s)
    b.commit()
    b.step(23, graph_steps=4)     # 5 graph replays + 3 direct steps
    st = b.sync()
    assert [int(x) for x in st[:len(GRIDS), 0]] == targets
    for k, g in enumerate(GRIDS):
        ref = _alone(lib, g, k, precision, flags, recon, targets[k])
        assert torch.equal(sol[k].distributions(), ref.distributions()), (k, g)
        assert torch.equal(sol[k].phi(), ref.phi()), (k, g)


def test_batch_admit_while_running(lib):
    """A grid attached after others have run: continuous batching."""
    import torch
    from paper_2007_07760_amd.batch import Batch
    print("case batch admit", flush=True)
    b = Batch(4, lib.F32, lib.UPWIND3, lib.FLAG_MASS_FIX)
    a = _solver(lib, GRIDS[1], 1, lib.F32, lib.FLAG_MASS_FIX, lib.UPWIND3)
    b.set(0, a, 20)
    b.commit()
    b.step(8, graph_steps=4)
    c = _solver(lib, GRIDS[3], 3, lib.F32, lib.FLAG_MASS_FIX, lib.UPWIND3)
    b.set(2, c, 12)
    b.commit()
    b.step(12, graph_steps=4)
    st = b.sync()
    assert int(st[0, 0]) == 20 and int(st[2, 0]) == 12
    # a grid that had stepped alone first, then joins at its own step count
    d = _solver(lib, GRIDS[0], 0, lib.F32, lib.FLAG_MASS_FIX, lib.UPWIND3).step(5)
    b.clear(0)
    b.set(1, d, 15)
    b.commit()
    b.step(10, graph_steps=0)
    b.sync()
    assert d.step_index == 15
    for s, g, k, n in ((a, GRIDS[1], 1, 20), (c, GRIDS[3], 3, 12), (d, GRIDS[0], 0, 15)):
        ref = _alone(lib, g, k, lib.F32, lib.FLAG_MASS_FIX, lib.UPWIND3, n)
        assert torch.equal(s.distributions(), ref.distributions()), g


def test_batch_tune_keeps_results(lib):
    import torch
    from paper_2007_07760_amd.batch import Batch
    print("case batch tune", flush=True)
    b = Batch(8, lib.F32, lib.UPWIND3, lib.FLAG_MASS_FIX)
    sol = []
    for k, g in enumerate(GRIDS):
        s = _solver(lib, g, k, lib.F32, lib.FLAG_MASS_FIX, lib.UPWIND3)
        b.set(k, s, 12)
        sol.append(s)
    b.commit()
    b.step(3, graph_steps=0)
    rows = b.tune(reps=2)
    assert rows % 8 == 0 and 16 <= rows <= 256 and b.tile_rows == rows
    b.step(9, graph_steps=3)
    b.sync()
    for k, g in enumerate(GRIDS):
        ref = _alone(lib, g, k, lib.F32, lib.FLAG_MASS_FIX, lib.UPWIND3, 12)
        assert torch.equal(sol[k].distributions(), ref.distributions()), (k, g)


def test_batch_rejects_mismatched_plan(lib):
    from paper_2007_07760_amd.batch import Batch
    b = Batch(2, lib.F32, lib.UPWIND3, lib.FLAG_MASS_FIX)
    s64 = _solver(lib, GRIDS[0], 0, lib.F64, 0, lib.UPWIND3)
    with pytest.raises(lib.DugksError):
        b.set(0, s64, 5)
    s32 = _solver(lib, GRIDS[0], 0, lib.F32, 0, lib.UPWIND3)   # no mass fix
    with pytest.raises(lib.DugksError):
        b.set(0, s32, 5)
    with pytest.raises(lib.DugksError):
        b.tile_rows = 12


def test_empty_batch_and_cleared_slots(lib):
    """A batch with no grid attached steps as a no-op (graph replays and
    single steps alike); a cleared slot stops advancing and keeps its state."""
    import torch
    from paper_2007_07760_amd.batch import Batch
    b = Batch(3, lib.F32, lib.UPWIND3, lib.FLAG_MASS_FIX)
    b.commit()
    b.step(5, graph_steps=2)
    st = b.sync()
    assert int(np.abs(st).sum()) == 0
    s = _solver(lib, GRIDS[1], 1, lib.F32, lib.FLAG_MASS_FIX, lib.UPWIND3)
    b.set(2, s, 100)
    b.commit()
    b.step(4)
    st = b.sync()
    assert int(st[2, 0]) == 4
    b.clear(2)
    b.commit()
    frozen = s.distributions().clone()
    b.step(3, graph_steps=3)
    b.sync()
    assert torch.equal(s.distributions(), frozen)
    ref = _alone(lib, GRIDS[1], 1, lib.F32, lib.FLAG_MASS_FIX, lib.UPWIND3, 4)
    assert torch.equal(frozen, ref.distributions())


@pytest.mark.parametrize("precision,flags", [(0, 0), (1, 0), (1, 2)])
def test_t3s3_batch_equals_alone(lib, precision, flags):
    """DUGKS-T3S3 grids in a DUGKS_BATCH_T3S3 batch (stage A and stage B
    kernels over all grids per batch step, graph replays) equal their alone
    runs bitwise, with targets that stop grids at different steps; FP32 also
    with the fused mass correction."""
    import torch
    from paper_2007_07760_amd.batch import Batch
    from paper_2007_07760_amd.solver import Solver

    def make(k, g):
        nx, ny, kind, prm = g
        return Solver(nx, ny, 0.02, 4.0, 0.5, recon=lib.UPWIND3, precision=precision,
                      vel_kind=kind, vel_param=prm, flags=flags,
                      scheme=lib.T3S3).init(_phi0(nx, ny, k))

    print(f"case T3S3 batch precision={precision} flags={flags}", flush=True)
    b = Batch(len(GRIDS), precision, lib.UPWIND3, lib.BATCH_T3S3 | flags)
    targets = [9 + 3 * k for k in range(len(GRIDS))]
    sol = []
    for k, g in enumerate(GRIDS):
        s = make(k, g)
        b.set(k, s, targets[k])
        sol.append(s)
    b.commit()
    b.step(max(targets), graph_steps=4)
    st = b.sync()
    for k, g in enumerate(GRIDS):
        assert int(st[k, 0]) == targets[k]
        ref = make(k, g).step(targets[k])
        assert torch.equal(sol[k].distributions(), ref.distributions()), (k, g)
    rows = b.tune(reps=1)
    assert rows > 0


def test_batch_scheme_must_match(lib):
    from paper_2007_07760_amd.batch import Batch
    from paper_2007_07760_amd.solver import Solver
    b = Batch(2, lib.F64, lib.UPWIND3, lib.BATCH_T3S3)
    t2 = Solver(40, 32, 0.02, 4.0, 0.5, recon=lib.UPWIND3).init(_phi0(40, 32, 0))
    with pytest.raises(lib.DugksError):
        b.set(0, t2, 5)
    b2 = Batch(2, lib.F64, lib.UPWIND3, 0)
    t3 = Solver(40, 32, 0.02, 4.0, 0.5, recon=lib.UPWIND3, scheme=lib.T3S3).init(_phi0(40, 32, 0))
    with pytest.raises(lib.DugksError):
        b2.set(0, t3, 5)


@pytest.mark.parametrize("precision,flags", [(1, 2), (0, 0)])
def test_batch_stops_a_blown_up_slot(lib, precision, flags):
    """A grid whose first state is non-finite is stopped after its first batch
    step with status ENUMERIC; the other grids run on, bitwise as alone."""
    import torch
    from paper_2007_07760_amd.batch import Batch
    from paper_2007_07760_amd.solver import Solver
    print(f"case batch blow-up prec={precision} flags={flags}", flush=True)
    b = Batch(4, precision, lib.UPWIND3, flags)
    good = []
    for k in (0, 1):
        s = _solver(lib, GRIDS[k], k, precision, flags, lib.UPWIND3)
        b.set(k, s, 16)
        good.append(s)
    nx, ny, kind, prm = GRIDS[3]
    phi0 = _phi0(nx, ny, 3)
    phi0[5, 7] = np.nan
    bad = Solver(nx, ny, 0.01, 4.0, 0.5, recon=lib.UPWIND3, precision=precision,
                 vel_kind=kind, vel_param=prm, flags=flags).init(phi0)
    b.set(2, bad, 16)
    b.commit()
    b.step(16, graph_steps=4)
    st = b.sync()
    status = b.status()
    assert list(status[:3]) == [lib.OK, lib.OK, lib.ENUMERIC]
    assert [int(x) for x in st[:3, 0]] == [16, 16, 1] and int(st[2, 1]) == 1
    for k, s in enumerate(good):
        ref = _alone(lib, GRIDS[k], k, precision, flags, lib.UPWIND3, 16)
        assert torch.equal(s.distributions(), ref.distributions()), k
    # a slot attached again after the failure starts with a clean status
    b.clear(2)
    c = _solver(lib, GRIDS[4], 4, precision, flags, lib.UPWIND3)
    b.set(2, c, 4)
    b.commit()
    assert b.status()[2] == lib.OK
    b.step(4, graph_steps=0)
    assert b.status()[2] == lib.OK and int(b.sync()[2, 0]) == 4


def test_batch_fused_correction_catches_a_blow_up_mid_run(lib):
    """FP32 with the fused correction: a grid whose state turns non-finite
    during the run is stopped at the next batch step by its own mass sum."""
    import torch
    from paper_2007_07760_amd.batch import Batch
    print("case batch blow-up mid-run", flush=True)
    b = Batch(2, lib.F32, lib.UPWIND3, lib.FLAG_MASS_FIX)
    a = _solver(lib, GRIDS[1], 1, lib.F32, lib.FLAG_MASS_FIX, lib.UPWIND3)
    z = _solver(lib, GRIDS[3], 3, lib.F32, lib.FLAG_MASS_FIX, lib.UPWIND3)
    b.set(0, a, 30)
    b.set(1, z, 30)
    b.commit()
    b.step(6, graph_steps=0)
    assert list(b.status()[:2]) == [lib.OK, lib.OK]
    n = z.state.numel()
    z.state[n // 4:3 * n // 4].view(torch.float32).fill_(float("nan"))
    b.step(24, graph_steps=4)
    st = b.sync()
    assert list(b.status()[:2]) == [lib.OK, lib.ENUMERIC]
    assert int(st[0, 0]) == 30 and int(st[1, 0]) == 7
    ref = _alone(lib, GRIDS[1], 1, lib.F32, lib.FLAG_MASS_FIX, lib.UPWIND3, 30)
    assert torch.equal(a.distributions(), ref.distributions())


def test_batch_refuses_velocity_arrays(lib):
    from paper_2007_07760_amd.batch import Batch
    from paper_2007_07760_amd.solver import Solver
    b = Batch(2, lib.F64, lib.UPWIND3, 0)
    uv = np.zeros((2, 32, 40))
    s = Solver(40, 32, 0.01, 4.0, 0.5, recon=lib.UPWIND3, vel_kind=lib.VEL_ARRAYS).init(
        _phi0(40, 32, 0), uv)
    with pytest.raises(lib.DugksError) as e:
        b.set(0, s, 5)
    assert e.value.code == lib.EUNSUPPORTED
