"""The CPU oracle against what the paper and mathematics fix (no GPU)."""
import pytest

import oracle_checks as C


@pytest.mark.parametrize("check", C.ALL_CHECKS, ids=lambda f: f.__name__)
def test_oracle_pin(check):
    check()


def test_golden_eddy_table_parses():
    rows = C.golden_eddies()
    assert len(rows) == 12
    assert {r["theta"] for r in rows} == {45.0, 60.0, 75.0}
    # the primary eddy moves right as n falls (Tables 1-3)
    for th in (45.0, 60.0, 75.0):
        xs = [r["primary"][0] for r in sorted((r for r in rows if r["theta"] == th), key=lambda r: -r["n"])]
        assert xs == sorted(xs)
