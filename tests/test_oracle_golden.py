"""Golden values printed in the paper."""
import csv
import os

import numpy as np

from oracle import operator as O

HERE = os.path.join(os.path.dirname(__file__), "golden")


def test_table1_g_ranges():
    """G = c / (f h) reproduces the G_m / G_M columns of Table 1 to the printed
    precision (the table-index selection uses this G)."""
    with open(os.path.join(HERE, "table1_g_range.csv")) as fh:
        rows = list(csv.DictReader(r for r in fh if not r.startswith("#")))
    assert len(rows) == 5
    for r in rows:
        f, h = float(r["f"]), float(r["h"])
        tol = 0.5 * 10 ** -int(r["printed_decimals"]) + 1e-9
        for c, g in ((float(r["c_m"]), float(r["G_m"])), (float(r["c_M"]), float(r["G_M"]))):
            # index selection on a table with spacing 0.01 starting at 0 returns G itself
            idx, _ = O.select_index(np.array([c], np.float32), f, h, 0.0, 0.01, 10000)
            assert abs(idx[0] * 0.01 - g) <= tol + 0.005, r["model"]
