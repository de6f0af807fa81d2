"""The oracle against the numbers the paper prints (Table I) and the
convergence order it reports.  Values depend on choices the paper leaves open
(stencils, tie rule, d(phi u)/dt), so they are soft pins with a stated
tolerance; the run is the paper's exact configuration."""
import json
import math
import os

import pytest

from paper_2007_07760_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_translation_n128.json")


def _translation(orc, n, recon, cfl, pe=128.0, cn=1 / 32, m=0.02):
    u0 = pe * m / n
    w = cn * n
    steps = int(round(n / u0 / cfl))
    phi0 = I.tanh_circle(n, n, n / 2, n / 2, n / 5, w)
    p = orc.Params(n, n, m, w, cfl, recon, 0, (u0, u0))
    s = orc.State(p, phi0).run(steps)
    return orc.e_phi(s.phi(), phi0)


@pytest.mark.parametrize("scheme,cfl", [("T2S3", 0.8), ("T2S2CD", 0.5)])
def test_table1_translation_n128(orc, scheme, cfl):
    rows = json.load(open(GOLDEN))["rows"]
    row = next(r for r in rows if r["scheme"] == scheme and r["cfl"] == cfl)
    e = _translation(orc, 128, row["recon"], cfl)
    # within 5 % of the printed value (the readings reproduce it to ~1 %)
    assert e == pytest.approx(row["E_phi"], rel=0.05), e


def test_second_order_convergence(orc):
    """Sec. III.A: every DUGKS variant converges at second order (Table I,
    ratio ~4 per doubling).  Pe = 128, Cn = 1/16 at L0 = 64 and 128."""
    e64 = _translation(orc, 64, 1, 0.8, cn=1 / 16)
    e128 = _translation(orc, 128, 1, 0.8, cn=1 / 16)
    order = math.log2(e64 / e128)
    assert 1.8 < order < 2.2, order
