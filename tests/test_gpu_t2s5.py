"""DUGKS-T2S5 (the fifth-order reconstruction of Sec. III) on the GPU against
the FP64 oracle's reading of it (ORC_UPWIND5).

The kernel runs the same march as the other T2 schemes with the wide patch:
a 6-row ring, faces three rows behind the cell terms, and the strip's edge
lanes computing phi one column further out.  Bar: FP64 relative L-inf
<= 1e-12, on trajectories and on single steps from the GPU's own state.  The
paper's T2S5 numbers are a comparison (its stencil is not printed), not a pin.
"""
import json
import os

import numpy as np
import pytest

from paper_2007_07760_amd import inputs as I
from test_gpu_parity import KINDS, _check, _pair, checkpoints_run

pytestmark = pytest.mark.gpu

UPWIND5 = 3


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2007_07760_amd import _lib
    _lib.load()
    from paper_2007_07760_amd.solver import Solver
    return Solver


@pytest.mark.parametrize("kind", range(4))
def test_t2s5_ragged(gpu, orc, kind):
    """100 x 72 (two strips, the second ragged), 16-row tiles, every velocity
    kind; then one step from the GPU state after 300 steps."""
    nx, ny = 100, 72
    phi0 = I.random_circles(nx, ny, 5, 6.0, 14.0, 4.0, seed=31 + kind)
    k, prm = KINDS[kind]
    g, o = _pair(gpu, orc, nx, ny, 0.01, 4.0, 0.6, UPWIND5, k, prm, phi0, tile_rows=16)
    for steps in (1, 2, 37):
        g.step(steps)
        o.run(steps)
        _check(g, o, f"t2s5 ragged +{steps}", orc)
    checkpoints_run(g, orc, o.p, (300,), "t2s5 ragged")


@pytest.mark.parametrize("shape,tile", [((8, 8), 0), ((8, 8), 1), ((58, 9), 3),
                                        ((59, 13), 5), ((40, 24), 7), ((130, 11), 64),
                                        ((17, 120), 2), ((64, 64), 9)])
def test_t2s5_edge_sizes(gpu, orc, shape, tile):
    """Grids narrower than a wavefront (the edge lanes' outer column wraps onto
    the grid), a ragged strip of one column, single-row segments, CFL 0.8."""
    nx, ny = shape
    phi0 = I.random_smooth(nx, ny, seed=nx * 3 + ny)
    g, o = _pair(gpu, orc, nx, ny, 0.02, 3.0, 0.8, UPWIND5, 1, (0.002, nx / 2, ny / 3),
                 phi0, tile_rows=tile)
    g.step(12)
    o.run(12)
    _check(g, o, "t2s5 edge", orc)


def test_t2s5_cfl_one_and_theta_off(gpu, orc):
    nx, ny = 64, 40
    phi0 = I.random_smooth(nx, ny, seed=6)
    g, o = _pair(gpu, orc, nx, ny, 0.03, float("inf"), 1.0, UPWIND5, 0, (0.05, -0.03),
                 phi0, tile_rows=9)
    g.step(20)
    o.run(20)
    _check(g, o, "t2s5 cfl 1, theta off", orc)


def test_t2s5_tile_shape_invariance_bitwise(gpu):
    nx, ny = 150, 97
    phi0 = I.random_circles(nx, ny, 6, 6.0, 20.0, 4.0, seed=8)
    for precision, flags in ((0, 0), (1, 2)):
        ref = None
        for tile in (0, 1, 5, 16, 33, 97):
            g = gpu(nx, ny, 0.01, 4.0, 0.5, recon=UPWIND5, precision=precision, flags=flags,
                    vel_kind=2, vel_param=(0.05, 400.0), tile_rows=tile).init(phi0)
            g.step(25)
            f = g.distributions().cpu().numpy()
            if ref is None:
                ref = f
            else:
                assert np.array_equal(f, ref), (precision, tile)


def test_t2s5_translation_full_period(gpu, orc):
    """The Table I case at N = 128 (Pe = 128, Cn = 1/32, M = 0.02, C = 0.5,
    12 800 steps): trajectory to step 400, one step from the GPU state at
    steps 3000, 8000 and 12 799, and E_phi beside the printed value."""
    from paper_2007_07760_amd import paper_runs as R
    c = R.translation(128, 128.0, 1 / 32, 0.02, 0.5, UPWIND5)
    phi0 = c["phi0"]()
    g, o = _pair(gpu, orc, c["nx"], c["ny"], c["mobility"], c["width"], c["cfl"], UPWIND5,
                 c["vel_kind"], c["vel_param"], phi0, twin=False)
    g.step(400)
    o.run(400)
    _check(g, o, "t2s5 N=128 step 400", orc)
    checkpoints_run(g, orc, o.p, (3000, 8000, c["steps"] - 1), "t2s5 N=128")
    e = R.e_phi(g.phi().cpu().numpy(), phi0)
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                       "paper_tables.json")))
    printed = gold["I"]["T2S5"]["CFL0.5"][0]
    print(f"T2S5 Table I N=128 C=0.5: E_phi {e:.4e}, printed {printed:.3e}, "
          f"ratio {e / printed:.3f}", flush=True)
    assert abs(e / printed - 1) < 0.05


def test_t2s5_headline_size_two_steps(gpu, orc):
    w = I.workload("h1")
    g, o = _pair(gpu, orc, w["nx"], w["ny"], w["mobility"], w["width"], w["cfl"], UPWIND5,
                 w["vel_kind"], w["vel_param"], w["phi0"], twin=False)
    g.step(2)
    o.run(2)
    _check(g, o, "t2s5 4096^2 step 2", orc)


def test_t2s5_fp32_mass_fix(gpu):
    """FP32 with the fused correction: drift <= 1e-9 on the slotted disk."""
    from paper_2007_07760_amd import _lib as C
    w = I.workload("c2")
    g = gpu(w["nx"], w["ny"], w["mobility"], w["width"], w["cfl"], recon=UPWIND5,
            precision=C.F32, flags=C.FLAG_MASS_FIX, vel_kind=w["vel_kind"],
            vel_param=w["vel_param"]).init(w["phi0"])
    m0 = g.mass0()
    for _ in range(4):
        g.step(250)
        assert abs(g.mass() - m0) / m0 <= 1e-9


def test_t2s5_refused_where_not_provided(gpu):
    from paper_2007_07760_amd import _lib as C
    for kw in (dict(scheme=C.T3S3, mobility=0.05), dict(vel_kind=C.VEL_ARRAYS)):
        p = C.make_params(64, 64, kw.pop("mobility", 0.01), 4.0, 0.5, UPWIND5, **kw)
        assert C.dugks_plan_create_status(p) == C.EUNSUPPORTED
    with pytest.raises(C.DugksError) as e:
        C.dugks_batch_create(4, C.F64, UPWIND5, 0)
    assert e.value.code == C.EUNSUPPORTED
