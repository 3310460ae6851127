"""Rayleigh-Benard cube: time-averaged Nusselt and Reynolds numbers and
dissipation rates (Sec. 4, Table 4), in one storage format or several.

    python -m paper_1903_08882_amd.rb --N 257 --Ra 1e7 --Pr 0.7 --storage fp32 fp16s

For each storage format: fluid at rest with seeded temperature noise, a
transient of at least `--min-transient` free-fall times, run in blocks of
`--block-tf` free-fall times until the block means of Nu_vol of two successive
blocks differ by less than `--settle` (relative), then `--avg-steps` steps of
averaging split into `--sub` equal sub-blocks, the observables sampled every
`--sample-every` steps and accumulated in FP64 on the GPU.  Reports the means,
the standard error of the sub-block means (or, with `--batches`, of the means of
that many runs of consecutive sub-blocks, which are less correlated than single
short sub-blocks), optionally the same over the first `--prefix-steps` averaging
steps, and the paper's values for the same
(Ra, Pr) as context (the paper's grids and averaging times differ).  One JSON
line per storage format, then a comparison line when there are several.
"""
import argparse
import json
import math
import time

import torch

from . import binding as B
from . import synth

# Sec. 4, Table 4: Re_rms, Re_w, Nu_vol, Nu_wall, Nu_kin, Nu_th.
PAPER = {
    (1e6, 0.7): (208.80, 145.58, 8.33, 8.35, 8.24, 8.26),
    (3e6, 0.7): (357.11, 249.96, 11.46, 11.48, 11.35, 11.37),
    (1e7, 0.7): (654.86, 454.92, 16.22, 16.27, 16.07, 16.10),
    (1e6, 7.0): (26.13, 20.26, 8.49, 8.52, 8.46, 8.44),
    (3e6, 7.0): (44.56, 33.65, 11.12, 11.14, 11.08, 11.06),
    (1e7, 7.0): (86.41, 65.71, 16.16, 16.19, 16.11, 16.03),
}
KEYS = ["Re_rms", "Re_w", "Nu_vol", "Nu_wall", "Nu_kin", "Nu_th", "eps_u", "eps_T",
        "Nu_hot", "Nu_cold", "Nu_hot_fd", "Nu_cold_fd"]


def _summary(params, raw):
    nd = B.lbm_nondimensional(params, raw)
    nd["Nu_wall"] = 0.5 * (nd["Nu_hot"] + nd["Nu_cold"])
    return {k: nd[k] for k in KEYS}


def standard_errors(subs, keys):
    """Standard error of the mean of each key over equal sub-blocks: the
    sample standard deviation of the sub-block values over sqrt(count); NaN
    for a single sub-block."""
    n = len(subs)
    out = {}
    for k in keys:
        if n < 2:
            out[k] = float("nan")
            continue
        m = sum(s[k] for s in subs) / n
        out[k] = math.sqrt(sum((s[k] - m) ** 2 for s in subs) / (n - 1) / n)
    return out


def _mean_raw(raws):
    return [sum(r[j] for r in raws) / len(raws) for j in range(len(raws[0]))]


def batch_means(params, raws, batches):
    """Group equal sub-blocks into `batches` runs of consecutive sub-blocks
    and summarise each run from its mean raw sums (the observables are ratios
    of the sums, so a run's value comes from its sums, not from averaging the
    sub-block ratios).  The count of sub-blocks must be a multiple of
    `batches`."""
    if batches <= 0 or len(raws) % batches:
        raise ValueError(f"{len(raws)} sub-blocks do not split into {batches} batches")
    g = len(raws) // batches
    return [_summary(params, _mean_raw(raws[i * g:(i + 1) * g])) for i in range(batches)]


def averaging_plan(avg_steps, sub, sample_every, batches=None, prefix_steps=None):
    """Steps per averaging sub-block (a whole number of sample intervals) and
    the number of leading sub-blocks the prefix covers (None without one).
    Raises ValueError, before anything runs, when `batches` does not divide
    `sub` or the prefix is not 2..sub whole sub-blocks."""
    per = max(sample_every, (avg_steps // sub) // sample_every * sample_every)
    if batches is not None and (batches <= 0 or sub % batches):
        raise ValueError(f"{sub} sub-blocks do not split into {batches} batches")
    k = None
    if prefix_steps:
        k = prefix_steps // per
        if k < 2 or k * per != prefix_steps or k > sub:
            raise ValueError(f"prefix of {prefix_steps} steps is not 2..{sub} sub-blocks of {per}")
    return per, k


def summarize_averages(params, raws, batches=None, k_prefix=None):
    """Means and standard errors of the averaging sub-blocks' raw sums: the
    mean from the pooled sums, the errors over `batches` runs of consecutive
    sub-blocks (or over the sub-blocks), and the same for the first
    `k_prefix` sub-blocks (errors over its sub-blocks)."""
    subs = [_summary(params, r) for r in raws]
    mean = _summary(params, _mean_raw(raws))
    se = standard_errors(batch_means(params, raws, batches) if batches else subs, KEYS)
    prefix = None
    if k_prefix:
        prefix = {"mean": _summary(params, _mean_raw(raws[:k_prefix])),
                  "stderr": standard_errors(subs[:k_prefix], KEYS)}
    return mean, se, prefix


def run_case(N, Ra, Pr, storage, seed, min_transient_tf=100.0, block_tf=20.0, settle=0.01,
             max_transient_tf=400.0, avg_steps=100_000, sub=10, sample_every=100, log=print,
             batches=None, prefix_steps=None):
    per, k_prefix = averaging_plan(avg_steps, sub, sample_every, batches, prefix_steps)
    opts = B.lbm_default_opts(sample_every=sample_every)
    h = B.lbm_create(N, Ra, Pr, "rayleigh_benard", storage, opts)
    p = B.lbm_get_params(h)
    tf = p.H / p.U                                   # steps per free-fall time
    blk = max(sample_every, int(round(block_tf * tf / sample_every)) * sample_every)
    B.lbm_set_fields(h, torch.from_numpy(synth.rest_with_noise(N, seed).reshape(-1)).cuda())
    t0 = time.perf_counter()
    steps, prev, trans, settled = 0, None, [], False
    while True:
        B.lbm_reset_averages(h)
        B.lbm_step(h, blk)
        raw, _ = B.lbm_averages(h)
        steps += blk
        nu = _summary(p, raw)["Nu_vol"]
        if not math.isfinite(nu):
            raise B.LBMError(-5, f"Nu_vol not finite after {steps} steps")
        trans.append(nu)
        d = abs(nu - prev) / abs(nu) if prev is not None else float("inf")
        log(f"# {storage} transient {steps} steps ({steps / tf:.0f} t_f): block Nu_vol {nu:.4f} "
            f"(change {d:.2%})  {time.perf_counter() - t0:.0f} s")
        prev = nu
        if steps >= min_transient_tf * tf and d < settle:
            settled = True
            break
        if steps >= max_transient_tf * tf:
            log(f"# {storage}: block means still moving after {max_transient_tf:.0f} t_f")
            break
    transient = steps
    subs, raws = [], []
    ta = time.perf_counter()
    for i in range(sub):
        B.lbm_reset_averages(h)
        B.lbm_step(h, per)
        raw, cnt = B.lbm_averages(h)
        raws.append(raw)
        subs.append(_summary(p, raw))
        log(f"# {storage} averaging {i + 1}/{sub}: Nu_vol {subs[-1]['Nu_vol']:.4f} "
            f"Re_rms {subs[-1]['Re_rms']:.2f}  {time.perf_counter() - t0:.0f} s")
    torch.cuda.synchronize()
    wall_avg = time.perf_counter() - ta
    mean, se, prefix = summarize_averages(p, raws, batches, k_prefix)
    out = {"N": N, "Ra": Ra, "Pr": Pr, "storage": storage, "seed": seed,
           "steps_per_tf": tf, "transient_steps": transient, "transient_block_Nu_vol": trans,
           "settled": settled,
           "avg_steps": per * sub, "avg_tf": per * sub / tf, "samples": per * sub // sample_every,
           "stderr_over": f"{batches or sub} batches of {sub // (batches or sub)} sub-blocks",
           "mean": mean, "stderr": se,
           "MLUPS_averaging": N ** 3 * per * sub / wall_avg / 1e6,
           "wall_s": time.perf_counter() - t0}
    if prefix:
        out["prefix"] = {"avg_steps": k_prefix * per, "avg_tf": k_prefix * per / tf, **prefix,
                         "stderr_over": f"{k_prefix} sub-blocks"}
    ref = PAPER.get((Ra, Pr))
    if ref:
        out["paper"] = dict(zip(KEYS[:6], ref))
    B.lbm_destroy(h)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--N", type=int, default=257)
    ap.add_argument("--Ra", type=float, default=1e7)
    ap.add_argument("--Pr", type=float, default=0.7)
    ap.add_argument("--storage", nargs="+", default=["fp32", "fp16s"],
                    choices=["fp32", "fp64", "fp16s", "fp16c"])
    ap.add_argument("--seed", type=int, default=None,
                    help="noise seed (default: base seed + 2 + case index)")
    ap.add_argument("--min-transient", type=float, default=100.0, help="free-fall times")
    ap.add_argument("--max-transient", type=float, default=400.0, help="free-fall times")
    ap.add_argument("--block-tf", type=float, default=20.0)
    ap.add_argument("--settle", type=float, default=0.01)
    ap.add_argument("--avg-steps", type=int, default=100_000)
    ap.add_argument("--sub", type=int, default=10)
    ap.add_argument("--sample-every", type=int, default=100)
    ap.add_argument("--batches", type=int, default=None,
                    help="standard errors over this many runs of consecutive sub-blocks "
                         "(default: over the sub-blocks themselves)")
    ap.add_argument("--prefix-steps", type=int, default=None,
                    help="also report the mean and standard error over the first this many "
                         "averaging steps (a whole number of sub-blocks)")
    a = ap.parse_args()
    cases = [(1e6, 0.7), (3e6, 0.7), (1e7, 0.7), (1e6, 7.0), (3e6, 7.0), (1e7, 7.0)]
    seed = a.seed
    if seed is None:
        idx = next((i for i, c in enumerate(cases) if c == (a.Ra, a.Pr)), 0)
        seed = synth.SEED0 + 2 + idx
    res = []
    for s in a.storage:
        r = run_case(a.N, a.Ra, a.Pr, s, seed, a.min_transient, a.block_tf, a.settle,
                     a.max_transient, a.avg_steps, a.sub, a.sample_every,
                     log=lambda m: print(m, flush=True), batches=a.batches,
                     prefix_steps=a.prefix_steps)
        res.append(r)
        print(json.dumps(r), flush=True)
    if len(res) > 1:
        base = res[0]
        print(json.dumps({"compare_against": base["storage"], "diff": compare(base, res[1:])}),
              flush=True)
        if a.prefix_steps:
            print(json.dumps({"compare_against": base["storage"], "over": "prefix",
                              "diff": compare(base["prefix"], [r["prefix"] | {"storage": r["storage"]}
                                                               for r in res[1:]])}), flush=True)


def compare(base, others):
    """Relative difference of each mean from `base`'s, with the two standard
    errors combined in quadrature relative to `base`'s mean."""
    cmp = {}
    for r in others:
        cmp[r["storage"]] = {
            k: {"rel_diff": (r["mean"][k] - base["mean"][k]) / base["mean"][k],
                "combined_stderr_rel": math.hypot(r["stderr"][k], base["stderr"][k])
                / abs(base["mean"][k])} for k in KEYS[:8]}
    return cmp


if __name__ == "__main__":
    main()
