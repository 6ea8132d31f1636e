"""The Fig. 2 measurement tool on a small lattice: every (l, N_s, form) runs
exactly Ml BiCG steps (forced freeze iterations), so the Mv counts are the
cost table's (2 M l for the single and pseudo-double pass, 4 M l for the
double pass, Section 3) whatever N_s, and the table has one row per
(l, N_s) with one time per form."""
import pytest

from tests.helpers import log

pytestmark = pytest.mark.gpu


def test_fig2_sweep_counts_and_table():
    from paper_1010_2592_amd import fig2_sweep as f2
    ls, ns_list, ml = [1, 2, 4], [2, 8], 16
    rho, rows = f2.sweep((4, 4, 4, 8), ml, ls, ns_list, 1, log=log)
    assert rho > 0
    assert len(rows) == len(ls) * len(ns_list) * len(f2.FORMS)
    for r in rows:
        M = ml // r["l"]
        assert r["status"] in (0, 4), r            # OK or NOT_CONVERGED (forced freeze)
        assert r["outer"] == M, r
        assert r["mv"] == (4 if r["pass"] == 2 else 2) * M * r["l"], r
        assert r["ms"] > 0
    tab = f2.table(rows, ls, ns_list).splitlines()
    assert len(tab) == 2 + len(ls) * len(ns_list)
    assert all(line.count("|") == 3 + len(f2.FORMS) for line in tab)
