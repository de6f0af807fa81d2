"""Host-side checks of the paper-table definitions (no GPU): every table's
configurations follow the parameters of Sec. III, and the T3S3 entries the
paper leaves empty are exactly those the scheme does not allow (dt >= 12 tau
with tau = 3 M) -- an independent pin of the reading tau = M / RT."""
import json
import math
import os

import pytest

from paper_2007_07760_amd import paper_runs as P

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))
TABLES = ["I", "II", "III", "IV", "V", "VIII", "IX"]


@pytest.mark.parametrize("table", TABLES)
def test_empty_entries_are_the_disallowed_ones(table):
    cols, cfgs = P.table_configs(table, "T3S3")
    g = GOLD[table]
    assert [float(c) for c in g["cols"]] == [float(c) for c in cols]
    for k, c in enumerate(cfgs):
        printed = g["T3S3"][f"CFL{P.CFLS[k // len(cols)]}"][k % len(cols)]
        assert (printed is None) == (not P.allowed(c)), (table, k)
    # the T2 variants have every entry
    for scheme in ("T2S2CD", "T2S3"):
        _, cf = P.table_configs(table, scheme)
        assert all(P.allowed(c) for c in cf)
        assert all(v is not None for row in g[scheme].values() for v in row)
    # T2S5 is a two-level scheme too: the paper prints every entry
    assert all(len(row) == len(cols) and None not in row for row in g["T2S5"].values())


@pytest.mark.parametrize("table", TABLES)
def test_table_parameters(table):
    """Pe = U0 L0 / M, Cn = W / L0 and the run length of Sec. III."""
    cols, cfgs = P.table_configs(table, "T2S3")
    assert len(cfgs) == 3 * len(cols)
    for k, c in enumerate(cfgs):
        n, m = c["nx"], c["mobility"]
        assert c["ny"] == n and c["cfl"] == P.CFLS[k // len(cols)]
        u0 = (math.hypot(*c["vel_param"][:2]) / math.sqrt(2) if c["kind"] == "translation"
              else (c["vel_param"][0] * n / math.pi if c["kind"] == "zalesak"
                    else c["vel_param"][0]))
        pe = u0 * n / m
        col = cols[k % len(cols)]
        if table in ("II", "IV", "VIII"):
            assert pe == pytest.approx(col)
        elif table in ("III", "V", "IX"):
            assert m == pytest.approx(col)
        else:
            assert n == col
        periods = 2.0 if c["kind"] == "zalesak" else 1.0
        assert c["steps"] == round(periods * n / u0 / c["cfl"])
