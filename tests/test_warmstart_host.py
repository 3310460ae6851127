"""Host-side logic of the warm-start driver (no GPU): the fall-back rule, the
Nu settling measure and the record of a run made in two precision stages."""
import math

import pytest

torch = pytest.importorskip("torch")
from paper_1903_08882_amd.warmstart import (keep_warm_start, merge_stages, steps_to_nu,  # noqa: E402
                                            strategy_cost)


def test_fallback_judges_the_warm_run_from_its_own_residual():
    """The rule sees only the warm run (causal): its residual after the probe
    (check 20 of 1000 steps each, index 19) against its first check."""
    decaying = [1e-2 * 0.8 ** j for j in range(40)]            # 1e-2 -> 1.4e-4 at the probe
    assert keep_warm_start(decaying, 1000, 20_000)
    assert not keep_warm_start(decaying, 1000, 20_000, decay=100.0)
    growing = [1e-4 * 1.1 ** j for j in range(40)]              # a start from rest: convection sets in
    assert not keep_warm_start(growing, 1000, 20_000)
    flat = [1e-3] * 40
    assert not keep_warm_start(flat, 1000, 20_000)
    assert keep_warm_start([1e-3, 1e-5, 1e-7], 1000, 20_000)   # met its tolerance before the probe
    assert not keep_warm_start([1e-3, math.nan], 1000, 20_000)
    assert not keep_warm_start([math.inf] + decaying, 1000, 20_000)
    assert not keep_warm_start(decaying[:19] + [math.nan] + decaying[20:], 1000, 20_000)
    assert not keep_warm_start([], 1000, 20_000)


def test_fallen_back_strategy_pays_the_probe():
    warm = {"steps": 150_000, "wall_s": 15.0, "probe": (20_000, 3e-3, 2.1)}
    cold = {"steps": 300_000, "wall_s": 30.0}
    assert strategy_cost(warm, cold, True) == (150_000, 15.0)
    assert strategy_cost(warm, cold, False) == (320_000, 32.1)


def test_steps_to_nu_counts_from_the_last_entry_into_the_band():
    ref = 10.0
    track = [(10, 8.0, 8.2), (20, 9.98, 10.1), (30, 10.2, 10.1), (40, 10.02, 9.99), (50, 10.01, 10.0)]
    assert steps_to_nu(track, ref, 5e-3, wall="hot") == 40      # 9.98 in, 10.2 out, back in at 40
    assert steps_to_nu(track, ref, 5e-3, wall="mean") == 40     # means 8.1, 10.04, 10.15, 10.005, 10.005
    assert steps_to_nu(track, ref, 1e-4, wall="hot") is None
    assert steps_to_nu([(5, 10.0)], ref) == 5                   # hot-only tracks


def test_two_stage_record_adds_steps_and_shifts_the_second_nu_track():
    r1 = {"steps": 68000, "max_dT": 9e-5, "converged": True, "wall_s": 3.0, "probe": (20000, 1e-2, 0.9),
          "history": [1e-2, 9e-5], "nu_track": [(20000, 9.0, 8.0), (68000, 8.7, 8.6)]}
    r2 = {"steps": 210000, "max_dT": 9e-9, "converged": True, "wall_s": 29.0, "probe": (1000, 8e-5, 0.1),
          "history": [8e-5, 9e-9], "nu_track": [(10000, 8.671, 8.670), (210000, 8.6708, 8.6708)]}
    r = merge_stages(r1, r2)
    assert r["steps"] == 278000 and r["wall_s"] == 32.0
    assert r["max_dT"] == 9e-9 and r["converged"]
    assert r["probe"] == (20000, 1e-2, 0.9)                         # the fall-back rule sees stage 1
    assert r["stage1"] == {"steps": 68000, "max_dT": 9e-5, "converged": True, "wall_s": 3.0}
    assert r["history"] == [1e-2, 9e-5, 8e-5, 9e-9]
    assert [row[0] for row in r["nu_track"]] == [20000, 68000, 78000, 278000]
    assert r["nu_track"][2] == (78000, 8.671, 8.670)
    assert steps_to_nu(r["nu_track"], 8.6708, 1e-3, wall="mean") == 78000
    assert r1["steps"] == 68000 and len(r1["nu_track"]) == 2       # inputs left unchanged
