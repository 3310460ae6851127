"""Host-side logic of the validation drivers (no GPU): three-grid Richardson
extrapolation, against a closed form and against the paper's own Table 2, and
the standard errors of the Rayleigh-Benard sub-block means."""
import math

import pytest

pytest.importorskip("torch")
from paper_1903_08882_amd.validate import PAPER, richardson  # noqa: E402


def test_richardson_recovers_a_power_law_exactly():
    for p_true in (1.0, 2.0, 3.5):
        ns = (81, 129, 257)
        fs = [5.0 + 3.0 * (1.0 / n) ** p_true for n in ns]
        p, finf = richardson(ns, fs)
        assert abs(p - p_true) < 1e-9 and abs(finf - 5.0) < 1e-9


def test_richardson_of_the_paper_table_2():
    """The paper's hot-wall Nu at Ra 1e6 on 81/129/161 converges with order
    2.14 to 8.6327, and at Ra 1e7 on 129/161/257 with order 1.94 to 16.318
    (the values quoted beside ours in the design notes)."""
    p, f = richardson((81, 129, 161), [PAPER[(n, 1e6)]["Nu_hot"] for n in (81, 129, 161)])
    assert abs(p - 2.14) < 0.01 and abs(f - 8.6327) < 1e-4
    p, f = richardson((129, 161, 257), [PAPER[(n, 1e7)]["Nu_hot"] for n in (129, 161, 257)])
    assert abs(p - 1.94) < 0.01 and abs(f - 16.3176) < 1e-4


def test_richardson_refuses_non_monotone_values():
    p, f = richardson((81, 129, 257), [1.0, 2.0, 1.5])
    assert math.isnan(p) and math.isnan(f)


def test_rayleigh_benard_standard_errors():
    import numpy as np
    from paper_1903_08882_amd.rb import standard_errors
    rng = np.random.default_rng(3)
    vals = rng.normal(16.0, 0.5, 10)
    se = standard_errors([{"Nu": v} for v in vals], ["Nu"])["Nu"]
    assert abs(se - np.std(vals, ddof=1) / np.sqrt(10)) < 1e-12
    assert math.isnan(standard_errors([{"Nu": 1.0}], ["Nu"])["Nu"])


def test_rayleigh_benard_batch_means_summarise_the_pooled_sums():
    """A batch's observables come from the mean of its sub-blocks' raw sums:
    one batch per sub-block gives the sub-block summaries, a single batch the
    summary of the pooled sums, and a count that does not split is refused."""
    import numpy as np
    from paper_1903_08882_amd import binding as B
    from paper_1903_08882_amd.rb import _summary, batch_means
    rng = np.random.default_rng(5)
    p = B.lbm_derive_params(33, 1e6, 0.7, 1)
    raws = []
    for _ in range(6):
        r = rng.uniform(1e-3, 1e-2, B.NRAW)
        raws.append(list(r))
    each = batch_means(p, raws, 6)
    for got, r in zip(each, raws):
        want = _summary(p, r)
        assert all(got[k] == want[k] for k in want)
    pooled = [sum(r[j] for r in raws) / 6 for j in range(B.NRAW)]
    one = batch_means(p, raws, 1)[0]
    want = _summary(p, pooled)
    assert all(abs(one[k] - want[k]) <= 1e-14 * abs(want[k]) for k in want)
    pairs = batch_means(p, raws, 3)
    want = _summary(p, [(a + b) / 2 for a, b in zip(raws[2], raws[3])])
    assert all(abs(pairs[1][k] - want[k]) <= 1e-14 * abs(want[k]) for k in want)
    with pytest.raises(ValueError):
        batch_means(p, raws, 4)


def test_rayleigh_benard_averaging_plan_refuses_bad_splits_before_running():
    from paper_1903_08882_amd.rb import averaging_plan
    assert averaging_plan(300_000, 30, 100, 10, 100_000) == (10_000, 10)
    assert averaging_plan(100_000, 10, 100) == (10_000, None)
    # sub-blocks are whole sample intervals
    assert averaging_plan(100_050, 10, 100)[0] == 10_000
    for bad in [dict(batches=7), dict(batches=0), dict(prefix_steps=10_000),
                dict(prefix_steps=105_000), dict(prefix_steps=400_000)]:
        with pytest.raises(ValueError):
            averaging_plan(300_000, 30, 100, **bad)


def test_rayleigh_benard_summary_of_sub_blocks():
    """The mean comes from the pooled sums; the prefix is the same summary of
    the leading sub-blocks; with every sub-block equal the errors vanish."""
    import numpy as np
    from paper_1903_08882_amd import binding as B
    from paper_1903_08882_amd.rb import KEYS, _summary, summarize_averages
    p = B.lbm_derive_params(33, 1e6, 0.7, 1)
    rng = np.random.default_rng(9)
    raws = [list(rng.uniform(1e-3, 1e-2, B.NRAW)) for _ in range(6)]
    mean, se, prefix = summarize_averages(p, raws, batches=3, k_prefix=2)
    pooled = _summary(p, [sum(r[j] for r in raws) / 6 for j in range(B.NRAW)])
    first2 = _summary(p, [(raws[0][j] + raws[1][j]) / 2 for j in range(B.NRAW)])
    for k in KEYS:
        assert abs(mean[k] - pooled[k]) <= 1e-14 * abs(pooled[k])
        assert abs(prefix["mean"][k] - first2[k]) <= 1e-14 * abs(first2[k])
        assert se[k] > 0 and prefix["stderr"][k] > 0
    same = [raws[0]] * 4
    _, se0, _ = summarize_averages(p, same, batches=2)
    assert all(se0[k] == 0 for k in KEYS)
    assert summarize_averages(p, raws)[2] is None
