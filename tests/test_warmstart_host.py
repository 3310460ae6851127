"""Host-side logic of the warm-start driver (no GPU): the fall-back rule and
the Nu settling measure."""
import math

import pytest

torch = pytest.importorskip("torch")
from paper_1903_08882_amd.warmstart import keep_warm_start, steps_to_nu  # noqa: E402


def test_fallback_keeps_warm_start_only_when_its_probe_residual_is_lower():
    assert keep_warm_start((20000, 1e-3), (20000, 1e-2))
    assert not keep_warm_start((20000, 1e-2), (20000, 1e-3))
    assert not keep_warm_start((20000, 1e-3), (20000, 1e-3))          # a tie keeps the cold start
    assert not keep_warm_start(None, (20000, 1e-3))
    assert not keep_warm_start((20000, math.nan), (20000, 1e-3))       # diverged warm start
    assert not keep_warm_start((20000, math.inf), (20000, 1e-3))
    assert keep_warm_start((20000, 1e-3), (20000, math.nan))           # diverged cold start


def test_steps_to_nu_counts_from_the_last_entry_into_the_band():
    ref = 10.0
    track = [(10, 8.0, 8.2), (20, 9.98, 10.1), (30, 10.2, 10.1), (40, 10.02, 9.99), (50, 10.01, 10.0)]
    assert steps_to_nu(track, ref, 5e-3, wall="hot") == 40      # 9.98 in, 10.2 out, back in at 40
    assert steps_to_nu(track, ref, 5e-3, wall="mean") == 40     # means 8.1, 10.04, 10.15, 10.005, 10.005
    assert steps_to_nu(track, ref, 1e-4, wall="hot") is None
    assert steps_to_nu([(5, 10.0)], ref) == 5                   # hot-only tracks
