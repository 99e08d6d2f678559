"""T_eff arithmetic against the numbers printed in the thesis (article 1)."""
import json
import os

from paper_2207_08716_amd import teff

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "teff_printed.json")))


def test_teff_printed_values():
    for c in GOLD["cases"]:
        got = teff.t_eff_gbs(c["n_cells"], c["p"], c["t_it"])
        assert abs(got - c["printed_gbs"]) <= c["rel_tol"] * c["printed_gbs"], (c["cite"], got)


def test_teff_382_cubed_matches_recomputation():
    # eq (39): (2*12+1) * 382^3 * 4 B * 1e-9 / 0.106 s
    assert 382 ** 3 == GOLD["cases"][0]["n_cells"]
    assert abs(teff.t_eff_gbs(382 ** 3, 4, 0.106) - 52.59) < 0.01


def test_parallel_efficiency_and_overhead():
    e = GOLD["efficiency"]
    assert abs(teff.parallel_efficiency(e["t_seq"], e["t_par"], e["P"]) - e["printed"]) < 5e-4
    o = GOLD["overhead"]
    assert abs(teff.overhead_share(o["overhead"], o["speedup"]) - o["printed"]) < 5e-4
    f = GOLD["fraction_of_peak"]
    assert round(100 * f["t_eff"] / f["t_peak"]) == f["printed_percent"]


def test_a_eff_counts():
    # 12 unknown + 1 known DOF (Table 1): 25 N p bytes per iteration
    assert teff.a_eff_bytes(10, 8) == 25 * 10 * 8
    assert teff.a_eff_bytes(511 ** 3, 8) == 25 * 511 ** 3 * 8
