"""The communication-volume model of the distributed algorithm against the
values Table 1 prints (tests/golden/table1_comm.json, cited there): the
wedge-checking column, the cover-edge column and the reductions of all
rows, and the two R-MAT rows the paper extrapolates."""
import json
import math
import os

import pytest

from paper_2210_00389_amd import comm_model as cm

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = json.load(open(os.path.join(HERE, "golden", "table1_comm.json")))

# Three significant digits in print: at most half a unit of the last digit.
PRINT_TOL = 0.005


def _rel(a, b):
    return abs(a / b - 1.0)


@pytest.mark.parametrize("r", TABLE["rows"], ids=lambda r: r["graph"])
def test_previous_column_is_two_ids_per_wedge(r):
    got = cm.wedge_volume_bits(r["n"], r["wedges"]) / 8
    assert _rel(got, cm.parse_bytes(r["previous"])) < PRINT_TOL


@pytest.mark.parametrize("r", TABLE["rows"], ids=lambda r: r["graph"])
def test_cover_column_real_graphs(r):
    """Every real-graph row is reproduced by the total-communication formula
    with 3 level bits (levels 0..7)."""
    got = cm.cover_volume_bits(r["n"], r["m"], r["k"], r["p"], level_bits=3) / 8
    assert _rel(got, cm.parse_bytes(r["this"])) < PRINT_TOL
    # no other level width fits every row: 2 and 4 bits miss by more than print rounding
    for lb in (2, 4):
        alt = cm.cover_volume_bits(r["n"], r["m"], r["k"], r["p"], level_bits=lb) / 8
        assert _rel(alt, cm.parse_bytes(r["this"])) > PRINT_TOL


# Two reduction cells disagree with their own row's volumes: loc-brightkite
# prints 20.4 where 26.5MB / 2.02MB = 13.1, soc-Epinions1 prints 10.7 where
# 86.7MB / 4.25MB = 20.4.  The volumes are taken as authoritative.
REDUCTION_CELL_OFF = {"loc-brightkite_edges", "soc-Epinions1"}


@pytest.mark.parametrize("r", TABLE["rows"], ids=lambda r: r["graph"])
def test_reduction_real_graphs(r):
    x = cm.row(r["graph"], r["n"], r["m"], r["k"], r["p"], 3, r["wedges"])
    printed_ratio = cm.parse_bytes(r["previous"]) / cm.parse_bytes(r["this"])
    assert _rel(x.reduction, printed_ratio) < 2 * PRINT_TOL
    if r["graph"] in REDUCTION_CELL_OFF:
        assert _rel(x.reduction, r["reduction"]) > 0.3
    else:
        # the printed ratio is of unrounded volumes, rounded to 3 digits
        assert _rel(x.reduction, r["reduction"]) < 2 * PRINT_TOL


@pytest.mark.parametrize("r", TABLE["rmat"], ids=lambda r: f"RMAT-{r['scale']}")
def test_rmat_rows(r):
    x = cm.rmat_row(r["scale"], r["p"], k=r["k"], wedges=r["wedges"], level_bits=r["level_bits"])
    assert (x.n, x.m) == (r["n"], r["m"])
    assert _rel(x.previous_bytes, cm.parse_bytes(r["previous"])) < PRINT_TOL
    # the table rounds 193.1 TiB down to "192TB"; 22.86 PiB prints as "22.8PB"
    assert _rel(x.cover_bytes, cm.parse_bytes(r["this"])) < 0.01
    assert _rel(x.reduction, r["reduction"]) < 0.01


def test_rmat_exact_totals():
    """The totals in bits, worked by hand from the formula: scale 36, p = 128,
    k = 0.311: 2^40 * (4 + (0.311 * 128 + 3) * 36) + 127 * 36."""
    v36 = cm.cover_volume_bits(2 ** 36, 2 ** 40, 0.311, 128, 4)
    assert v36 == pytest.approx(2 ** 40 * (4 + (0.311 * 128 + 3) * 36) + 127 * 36)
    assert v36 / 8 / 2 ** 40 == pytest.approx(193.136, abs=1e-3)  # TiB
    v42 = cm.cover_volume_bits(2 ** 42, 2 ** 46, 0.260, 256, 4)
    assert v42 / 8 / 2 ** 50 == pytest.approx(22.856, abs=1e-3)  # PiB


def test_fits():
    # k fit: 0.260 at scale 42 as printed; at scale 36 the fit gives 0.322
    # while the table uses 0.311 (the table's volume follows its own k)
    assert cm.k_fit(42) == pytest.approx(0.260, abs=5e-4)
    assert cm.k_fit(36) == pytest.approx(0.3221, abs=5e-4)
    assert cm.triangles_fit(2 ** 36) == pytest.approx(1.2e14, rel=0.01)
    assert cm.triangles_fit(2 ** 42) == pytest.approx(1.3e16, rel=0.01)


def test_parts_sum_to_total():
    parts = cm.cover_volume_parts_bits(5000, 20000, 0.4, 8, 3)
    assert sum(parts.values()) == pytest.approx(cm.cover_volume_bits(5000, 20000, 0.4, 8, 3))
    # one processor: the exchange term is k*m ids, no reduction traffic
    one = cm.cover_volume_parts_bits(1024, 100, 0.5, 1, 2)
    assert one["reduce"] == 0 and one["exchange"] == 0.5 * 100 * 10


def test_wedges_closed_forms():
    assert cm.wedges_from_degrees([5] + [1] * 5) == 10          # star K_{1,5}: C(5,2)
    assert cm.wedges_from_degrees([4] * 5) == 5 * 6              # K_5: 5 * C(4,2)
    assert cm.wedges_from_degrees([1] + [2] * 8 + [1]) == 8      # path of 10 vertices
    assert cm.wedges_from_degrees([]) == 0


def test_volume_for_count():
    x = cm.volume_for_count(n=1 << 20, m=15_700_000, h=8_744_317, num_levels=6, p=8)
    assert x.k == pytest.approx(8_744_317 / 15_700_000)
    assert x.level_bits == 3
    assert x.cover_bytes * 8 == pytest.approx(cm.cover_volume_bits(1 << 20, 15_700_000, x.k, 8, 3))
    with pytest.raises(ValueError):
        cm.volume_for_count(n=10, m=0, h=0, num_levels=1, p=2)


def test_units_round_trip():
    for s in ("526KB", "2.78MB", "1.03GB", "192TB", "22.8PB", "52.8EB"):
        assert cm.fmt_bytes(cm.parse_bytes(s)) == s
    assert math.isclose(cm.parse_bytes("1KB"), 1024)


@pytest.mark.parametrize("scale", [10, 20, 22])
def test_measured_k_near_the_fit(scale):
    """k = |H| / m of the seeded R-MAT graphs (the oracle's stored values)
    lies within 10% below to 5% above the paper's fit, which came from
    arbitrary roots on other R-MAT instances: a plausibility band, not a pin."""
    p = os.path.join(HERE, "golden", f"rmat_s{scale}.json")
    if not os.path.exists(p):
        pytest.skip("golden file not generated")
    g = json.load(open(p))
    ratio = (g["h"] / g["m"]) / cm.k_fit(scale)
    assert 0.90 <= ratio <= 1.05
