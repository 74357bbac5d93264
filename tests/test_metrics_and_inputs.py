"""Host-side logic: the paper's SYPD arithmetic against its own Table 1, the
cell-count convention, and the seeded input generators."""
import csv
import math
import os

import numpy as np
import pytest

from paper_2309_06662_amd import inputs, metrics

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_wall_time_per_step.csv")


def _rows():
    with open(GOLDEN) as f:
        lines = [l for l in f if not l.startswith("#")]
    return list(csv.DictReader(lines))


def _digits_halfwidth(text):
    """Half a unit in the last printed digit of a decimal string."""
    if "." in text:
        return 0.5 * 10.0 ** (-len(text.split(".")[1]))
    return 0.5


@pytest.mark.parametrize("row", _rows(), ids=lambda r: r["model"] + "_" + r["devices"].replace(" ", ""))
def test_sypd_formula_reproduces_table1(row):
    dt = float(row["dt"])
    wall = float(row["wall"])
    hw = _digits_halfwidth(row["wall"])
    lo, hi = metrics.sypd(dt, wall + hw), metrics.sypd(dt, wall - hw)
    printed = float(row["sypd"])
    phw = _digits_halfwidth(row["sypd"])
    overlap = (printed + phw >= lo) and (printed - phw <= hi)
    assert overlap == bool(int(row["consistent"])), (lo, hi, printed)


def test_cell_count_convention_matches_table1_grid_sizes():
    # Table 1 grid sizes are nx*ny*nz of the full lat-lon grid, land included:
    # R12 at 1/12 deg over 75S-75N with 48 levels, R48 at 1/48 deg with 100 levels
    assert abs(4320 * 1800 * 48 - 3.7e8) / 3.7e8 < 0.01
    assert abs(17280 * 7200 * 100 - 1.24e10) / 1.24e10 < 0.01
    assert metrics.cell_updates_per_second(10, 20, 30, 5, 2.0) == 10 * 20 * 30 * 5 / 2.0


def test_abstract_aquaplanet_rate():
    # abstract: 488 m at 15 simulated days per day is 0.04 SYPD
    assert abs(15.0 / 365.0 - 0.041) < 0.001


def test_splitmix64_reference_output():
    # splitmix64 seeded with 0 returns mix64(GOLDEN) first: 0xE220A8397B1DCDAF
    z = inputs._mix64(np.array([inputs.GOLDEN], dtype=np.uint64))[0]
    assert int(z) == 0xE220A8397B1DCDAF


def test_counter_rng_is_deterministic_and_normal():
    n = np.arange(200000, dtype=np.uint64)
    a = inputs.normal(3, inputs.STREAM_TEMPERATURE, n)
    b = inputs.normal(3, inputs.STREAM_TEMPERATURE, n)
    assert np.array_equal(a, b)
    assert abs(a.mean()) < 0.01 and abs(a.std() - 1.0) < 0.01
    # any element can be drawn on its own
    assert inputs.normal(3, 0, np.array([12345], dtype=np.uint64))[0] == a[12345]
    c = inputs.normal(3, inputs.STREAM_BATHYMETRY, n)
    assert abs(np.corrcoef(a, c)[0, 1]) < 0.01


def test_workload_inputs_shapes_and_ranges():
    w = inputs.LATLON_QUARTER.replace(nx=144, ny=60, nz=10, dx=2.5, dy=160.0 / 60)
    inp = inputs.make_inputs(w)
    assert inp["T0"].shape == (10, 60, 144)
    kb = inp["kbottom"]
    assert kb.dtype == np.int32 and kb.min() >= 0 and kb.max() <= 10
    assert (kb == 0).any() and (kb == 10).any()
    # the ridges rise to the surface north of 50S at 0 and 90 E
    lat = w.y0 + (np.arange(w.ny) + 0.5) * w.dy
    north = lat > -45
    d = inputs.seafloor_depth(w)
    assert np.all(d[north, 0] < 0.2 * w.depth) and np.all(d[north, 36] < 0.2 * w.depth)
    # circumpolar channel south of the ridges has open water at the ridge longitudes
    assert np.any(kb[lat < -55, 0] > 0)
    taux, tauy = inputs.wind_stress(w)
    assert np.allclose(taux[:, 0], 0.1 * np.cos(np.radians(lat)))
    assert np.all(tauy == 0)
    zc = inputs.layer_centre_z(w)
    assert np.isclose(zc[-1], -w.depth / w.nz / 2) and np.isclose(zc[0], -w.depth + w.depth / w.nz / 2)
