"""Wall-unit bookkeeping against the paper's Table "stats" (Sec. 4)."""

import math
import os

import pytest

from paper_2306_12739_amd.units import wall_units, re_tau_from_wall_shear

ROWS = [l.split() for l in open(os.path.join(os.path.dirname(__file__), "golden",
                                             "paper_table_stats_wall_units.txt"))
        if l.strip() and not l.startswith("#")]


@pytest.mark.parametrize("row", ROWS, ids=[r[0] for r in ROWS])
def test_table_stats_wall_units(row):
    lx, lz, nx, nz, my = float(row[1]), float(row[2]), int(row[3]), int(row[4]), int(row[5])
    re_tau = float(row[6])
    expect = dict(zip(["Lx+", "Ly+", "Lz+", "dx+", "dz+", "dywall+", "dycentre+"], map(float, row[7:])))
    got = wall_units(re_tau, lx * math.pi, lz * math.pi, nx, nz, my)
    for k, v in expect.items():
        # the table rounds to the printed digits
        digits = len(row[7 + list(expect).index(k)].split(".")[1])
        assert abs(got[k] - v) <= 0.5 * 10 ** (-digits) + 1e-9, (k, got[k], v)


def test_re_tau_from_laminar_channel():
    # laminar channel: dU/dy = 2 at the wall, Re_tau = sqrt(2 Re)
    assert abs(re_tau_from_wall_shear(4200.0, 2.0) - math.sqrt(8400.0)) < 1e-12
