"""The single-grid tile autotuner (dugks_tune) through the C ABI: it picks a
height from its candidate set, leaves the state (and the fused correction's
header) unchanged, and the steps after it equal those of the untuned plan
bitwise (results do not depend on the tiling)."""
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


@pytest.mark.parametrize("precision,flags,scheme,mobility", [
    (0, 0, 0, 0.005),   # FP64 T2
    (1, 2, 0, 0.005),   # FP32 with the fused mass correction
    (0, 0, 1, 0.02),    # FP64 T3S3 (dt < 12 tau)
    (1, 2, 1, 0.02),    # FP32 T3S3 with the fused mass correction
])
def test_tune_keeps_state_and_results(lib, precision, flags, scheme, mobility):
    import torch
    from paper_2007_07760_amd.solver import Solver
    w = I.workload("c2")
    print(f"tune case prec={precision} flags={flags} scheme={scheme}", flush=True)

    def make():
        return Solver(w["nx"], w["ny"], mobility, w["width"], w["cfl"], recon=w["recon"],
                      precision=precision, vel_kind=w["vel_kind"], vel_param=w["vel_param"],
                      flags=flags, scheme=scheme).init(w["phi0"]).step(7)

    a, b = make(), make()
    before = b.distributions().clone()
    m_before = b.mass()
    rows = b.tune(reps=1)
    print(f"tuned tile height {rows}", flush=True)
    assert rows == b.params.tile_rows
    assert 8 <= rows <= 256
    assert torch.equal(b.distributions(), before)
    assert b.mass() == m_before
    a.step(5)
    b.step(5)
    assert torch.equal(a.distributions(), b.distributions())
