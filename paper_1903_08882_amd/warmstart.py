"""Learned warm start of the steady side-heated cavity: train the encoder-decoder
(include/lws.h) on steady fields from the batched sweep, then start lattice
Boltzmann runs from its prediction and measure steps to steady state against a
start from rest.

    python -m paper_1903_08882_amd.warmstart train --out params.npz
    python -m paper_1903_08882_amd.warmstart compare --params params.npz --N 257 --Ra 1e7 \
        --symmetrize --cold-storage fp32 --ref-nu 16.3927

train: the 64-cavity sweep (``sweep.run_sweep``: N in {33, 49, 65}, Ra
log-uniform on [1e4, 1e7], Pr in {0.71, 7}, each resampled to M^3 = 65^3),
the last `--holdout` cavities held out; Adam on the mean squared error of the
nondimensional fields (u/U, v/U, w/U, T/dT).  Prints the loss curve and writes
the FP32 parameters.

compare: for one cavity, a cold run (rest + seeded noise) and a warm run (the
network's prediction interpolated onto the lattice) advance with the steady-
state check (max |dT| over `--check` steps) to `--tol`.  The warm run judges
itself: at `--probe` steps its residual must have fallen `--decay` times below
its residual at the first check (a start near the steady state relaxes from
the first check on); otherwise the prediction is dropped for a start from
rest in the same storage, and that strategy is charged the probe's steps and
time on top of the cold run's (fall back).  Reports steps, wall time, the
hot-wall Nusselt numbers of both runs and their relative difference, and the
reference value when given.
The warm run's storage defaults to FP16C (the customised 16-bit format);
`--cold-storage fp32` makes the cold run the plain FP32 method.
"""
import argparse
import json
import math
import time

import numpy as np
import torch

from . import binding as B
from . import lws as L
from . import synth

CH = (16, 32, 64)
M_DEFAULT = 65


def init_params(ch=CH, seed=synth.SEED0 + 7):
    """He-uniform convolution weights, zero FiLM and bias terms except a
    small random FiLM so the conditioning reaches every layer."""
    c1, c2, c3 = ch
    layers = [(8, c1, True), (c1, c1, True), (c1, c2, True), (c2, c2, True), (c2, c3, True),
              (c3, c3, True), (c3 + c2, c2, True), (c2 + c1, c1, True), (c1, 8, False)]
    out = []
    for k, (ci, co, film) in enumerate(layers):
        a = math.sqrt(6.0 / (27 * ci))
        if not film:
            a *= 0.1                                   # small initial output
        out.append(a * synth.uniform(seed, 2 * k, 27 * ci * co))
        if film:
            g = 0.05 * synth.uniform(seed, 2 * k + 1, 6 * co)
            out.append(g)
        else:
            out.append(np.zeros(co))
    return np.concatenate(out).astype(np.float32)


def _scales(cavities):
    """Per-cavity factors turning lattice fields into u/U and T/dT."""
    rows = []
    for c in cavities:
        p = B.lbm_derive_params(c["N"], c["Ra"], c["Pr"], "side_heated", "fp32")
        rows.append([1.0 / p.U] * 3 + [1.0 / p.dT])
    return np.array(rows)


def train(fields, cavities, iters=1500, batch=8, lr=2e-3, holdout=8, seed=synth.SEED0 + 8,
          ch=CH, log=print):
    """Adam on the sweep fields [K, 4, M, M, M] (FP32, GPU).  Returns (net, history)."""
    K, M = fields.shape[0], fields.shape[-1]
    net = L.lws_net_create(M, batch, ch)
    L.lws_net_set_params(net, init_params(ch))
    ra_pr = np.array([[c["Ra"], c["Pr"]] for c in cavities])
    scale = _scales(cavities)
    tr = np.arange(K - holdout)
    ho = np.arange(K - holdout, K)
    rng = np.random.default_rng(seed)
    hist = []
    t0 = time.perf_counter()
    order = []
    for it in range(1, iters + 1):
        if len(order) < batch:
            order += list(rng.permutation(tr))
        idx, order = order[:batch], order[batch:]
        tgt = fields[torch.as_tensor(idx, device=fields.device)].contiguous().view(-1)
        loss = L.lws_net_loss_grad(net, ra_pr[idx], tgt, scale[idx])
        lr_t = lr * (0.05 + 0.95 * 0.5 * (1 + math.cos(math.pi * (it - 1) / iters)))
        L.lws_net_adam(net, lr_t)
        if it % 50 == 0 or it == 1 or it == iters:
            hl = []
            for s in range(0, len(ho), batch):
                h = ho[s:s + batch]
                th = fields[torch.as_tensor(h, device=fields.device)].contiguous().view(-1)
                hl.append(L.lws_net_loss_grad(net, ra_pr[h], th, scale[h]) * len(h))
            hold = sum(hl) / len(ho) if len(ho) else float("nan")
            hist.append({"iter": it, "train_loss": loss, "holdout_loss": hold, "lr": lr_t,
                         "s": time.perf_counter() - t0})
            log(f"# iter {it}: train {loss:.4e}  holdout {hold:.4e}  lr {lr_t:.2e}  "
                f"{time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    return net, hist


def predict_fields(net, N, Ra, Pr, cell="side_heated", opts=None, symmetrize=False):
    """The network's fields for (Ra, Pr), interpolated onto the N^3 lattice (FP64
    [4 N^3]); with symmetrize, averaged over the steady cell's symmetries."""
    p = B.lbm_derive_params(N, Ra, Pr, cell, "fp32", opts)
    pred = L.lws_net_forward(net, [[Ra, Pr]])
    return L.lws_upsample_fields(pred, net.M, 8, N, cell, p.U, p.T_hot, p.T_cold, symmetrize=symmetrize)


def _run(h, check, tol, max_steps, probe, log, tag, chunk_checks=10):
    """Steady-state loop in chunks (the first ends at the probe step); returns
    steps, final residual, wall time, the residual at the probe, the residual
    history and the hot-wall Nu after every chunk."""
    steps, r, hist, nu = 0, float("inf"), [], []
    t0 = time.perf_counter()
    at_probe = None
    while steps < max_steps and not r < tol:
        n = probe - steps if steps < probe else chunk_checks * check
        n = max(check, min(n, max_steps - steps))
        k, r, hh = B.lbm_run_to_steady(h, check, tol, n, history_len=n // check + 1)
        steps += k
        hist += hh
        if at_probe is None and (steps >= probe or r < tol):
            at_probe = (steps, r, time.perf_counter() - t0)
        o = _nu(h)
        nu.append((steps, o["Nu_hot"], o["Nu_cold"]))
        log(f"# {tag}: step {steps}  max_dT {r:.3e}  Nu_hot {o['Nu_hot']:.4f}  Nu_cold {o['Nu_cold']:.4f}  "
            f"{time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    return {"steps": steps, "max_dT": r, "converged": r < tol, "wall_s": time.perf_counter() - t0,
            "probe": at_probe, "history": hist, "nu_track": nu}


def keep_warm_start(history, check, probe, decay=10.0):
    """The fall-back rule, decided from the warm run alone (causal): keep the
    warm start if its steady-state residual (max |dT| over one check interval,
    history[j] after (j + 1) check steps) has fallen at least `decay` times
    below its first value by the probe step, or if the run met its tolerance
    before the probe.  A prediction close to the steady state relaxes from
    the first check on; a start that sets off a transient (or diverges) does
    not.  A residual that is not a finite number never passes."""
    if not history:
        return False
    j = max(probe // check - 1, 0)
    first = history[0]
    if not math.isfinite(first):
        return False
    if j >= len(history):                  # converged before the probe
        return all(math.isfinite(v) for v in history)
    r = history[j]
    return math.isfinite(r) and r * decay <= first


def strategy_cost(warm, fallback, kept):
    """Steps and seconds the warm-start strategy costs: the warm run when
    kept; otherwise its probe (steps and time up to the probe) plus the
    fall-back run from rest."""
    if kept:
        return warm["steps"], warm["wall_s"]
    pst, _, pwall = warm["probe"] if warm.get("probe") else (0, None, 0.0)
    return pst + fallback["steps"], pwall + fallback["wall_s"]


def steps_to_nu(track, ref, rel=5e-3, wall="hot"):
    """First step after which the tracked hot-wall Nu (wall="hot") or the mean
    of the hot- and cold-wall Nu (wall="mean") stays within rel of ref (None
    if never)."""
    first = None
    for row in track:
        st = row[0]
        v = row[1] if wall == "hot" or len(row) < 3 else 0.5 * (row[1] + row[2])
        if abs(v - ref) <= rel * abs(ref):
            if first is None:
                first = st
        else:
            first = None
    return first


def _nu(h):
    nd = B.lbm_nondimensional(B.lbm_get_params(h), B.lbm_observables_raw(h))
    return {k: nd[k] for k in ("Nu_hot", "Nu_cold", "Nu_hot_mid", "Nu_hot_fd", "Re_rms")}


def _finish(h, N, Ra, Pr, r, finish_storage, check, finish_tol, max_steps, log, tag):
    """Second stage: carry the populations of h into a handle in
    finish_storage and continue to finish_tol; steps, wall time and the Nu
    track of both stages are added up."""
    pop = B.lbm_get_populations(h)
    h2 = B.lbm_create(N, Ra, Pr, "side_heated", finish_storage)
    B.lbm_set_populations(h2, pop)
    del pop
    r2 = _run(h2, check, finish_tol, max(max_steps - r["steps"], check), 0, log, f"{tag}/{finish_storage}")
    return h2, merge_stages(r, r2)


def merge_stages(r1, r2):
    """One run record from two consecutive stages: steps and wall time add
    up, the residual and convergence are the second stage's, the probe stays
    the first stage's, the residual histories are concatenated and the second
    stage's Nu track is shifted by the first stage's steps.  The first stage's
    own figures are kept under "stage1"."""
    r = dict(r1)
    r["stage1"] = {k: r1[k] for k in ("steps", "max_dT", "converged", "wall_s")}
    r["steps"] = r1["steps"] + r2["steps"]
    r["wall_s"] = r1["wall_s"] + r2["wall_s"]
    r["max_dT"], r["converged"] = r2["max_dT"], r2["converged"]
    r["history"] = list(r1["history"]) + list(r2["history"])
    r["nu_track"] = list(r1["nu_track"]) + [(st + r1["steps"],) + tuple(v) for st, *v in r2["nu_track"]]
    return r


def compare(net, N, Ra, Pr, storage="fp16c", check=1000, tol=1e-4, max_steps=2_000_000, probe=20_000,
            seed=synth.SEED0 + 1, ref_nu=None, cold_storage=None, runs=None, symmetrize=False,
            finish_storage=None, finish_tol=None, decay=10.0, log=print):
    """Cold start in cold_storage (default: storage) against the warm start in
    storage; with a cold_storage other than storage, a cold start in storage
    is run as well ("cold_same") to separate the two effects.  With
    finish_storage, every run continues from its state at tol in that storage
    to finish_tol (e.g. a 16-bit stage to 1e-4, then FP64 to 1e-8)."""
    cold_storage = cold_storage or storage
    out = {"N": N, "Ra": Ra, "Pr": Pr, "storage": storage, "cold_storage": cold_storage, "check": check,
           "tol": tol, "probe": probe, "symmetrize": symmetrize, "finish_storage": finish_storage,
           "finish_tol": finish_tol}
    res = {}
    plan = [("cold", cold_storage), ("warm", storage)]
    if cold_storage != storage:
        plan.append(("cold_same", storage))
    if runs:
        plan = [x for x in plan if x[0] in runs]
    for tag, st in plan:
        h = B.lbm_create(N, Ra, Pr, "side_heated", st)
        if tag != "warm":
            B.lbm_set_fields(h, torch.from_numpy(synth.rest_with_noise(N, seed).reshape(-1)).cuda())
        else:
            B.lbm_set_fields(h, predict_fields(net, N, Ra, Pr, symmetrize=symmetrize))
            # one step so the wall flux is defined, then the prediction's own Nu
            B.lbm_step(h, 1)
            out["predicted_Nu"] = _nu(h)
        r = _run(h, check, tol, max_steps, probe, log, tag)
        if finish_storage:
            h_next, r = _finish(h, N, Ra, Pr, r, finish_storage, check, finish_tol, max_steps, log, tag)
            B.lbm_destroy(h)
            h = h_next
        r["Nu"] = _nu(h)
        r["MLUPS"] = N ** 3 * r["steps"] / r["wall_s"] / 1e6
        r["storage"] = st
        if ref_nu:
            r["steps_to_Nu_within_0.5pct_of_ref"] = steps_to_nu(r["nu_track"], ref_nu)
            r["steps_to_mean_Nu_within_0.5pct_of_ref"] = steps_to_nu(r["nu_track"], ref_nu, wall="mean")
        res[tag] = r
        B.lbm_destroy(h)
        log(json.dumps({"run": tag, **{k: v for k, v in r.items() if k not in ("history",)}}))
    if "cold" not in res or "warm" not in res:
        return {**out, "runs": {t: {k: v for k, v in r.items() if k != "history"} for t, r in res.items()}}
    cold, warm = res["cold"], res["warm"]
    if "cold_same" in res:
        out["cold_same"] = {k: v for k, v in res["cold_same"].items() if k != "history"}
    # fall back: the warm run keeps going only if its own residual has decayed
    # by the probe; otherwise the strategy pays the probe and a start from rest
    # in the same storage
    base = res.get("cold_same", cold)
    keep = keep_warm_start(warm["history"], check, probe, decay)
    st_steps, st_wall = strategy_cost(warm, base, keep)
    out.update({"cold": {k: v for k, v in cold.items() if k != "history"},
                "warm": {k: v for k, v in warm.items() if k != "history"},
                "kept_warm_start": keep,
                "strategy_steps": st_steps, "strategy_wall_s": st_wall,
                "steps_saved": cold["steps"] - st_steps,
                "speedup_steps": cold["steps"] / max(st_steps, 1),
                "speedup_wall": cold["wall_s"] / max(st_wall, 1e-9),
                "Nu_rel_diff_warm_vs_cold": (warm["Nu"]["Nu_hot"] - cold["Nu"]["Nu_hot"]) / cold["Nu"]["Nu_hot"],
                "cold_history_every_10": cold["history"][::10],
                "warm_history_every_10": warm["history"][::10],
                "cold_history_head": cold["history"][:20],
                "warm_history_head": warm["history"][:20]})
    if ref_nu:
        out["ref_Nu_hot"] = ref_nu
        out["Nu_rel_diff_vs_ref"] = {t: (res[t]["Nu"]["Nu_hot"] - ref_nu) / ref_nu for t in res}
    return out


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--K", type=int, default=64)
    t.add_argument("--M", type=int, default=M_DEFAULT)
    t.add_argument("--sweep-steps", type=int, default=200_000)
    t.add_argument("--iters", type=int, default=1500)
    t.add_argument("--batch", type=int, default=8)
    t.add_argument("--lr", type=float, default=2e-3)
    t.add_argument("--holdout", type=int, default=8)
    t.add_argument("--out", default="")
    c = sub.add_parser("compare")
    c.add_argument("--params", required=True)
    c.add_argument("--N", type=int, default=257)
    c.add_argument("--Ra", type=float, default=1e7)
    c.add_argument("--Pr", type=float, default=0.71)
    c.add_argument("--storage", default="fp16c", choices=["fp32", "fp64", "fp16s", "fp16c"])
    c.add_argument("--cold-storage", default=None, choices=["fp32", "fp64", "fp16s", "fp16c"])
    c.add_argument("--check", type=int, default=1000)
    c.add_argument("--tol", type=float, default=1e-4)
    c.add_argument("--probe", type=int, default=20_000)
    c.add_argument("--decay", type=float, default=10.0,
                   help="keep the warm start if its residual fell this many times by the probe")
    c.add_argument("--max-steps", type=int, default=2_000_000)
    c.add_argument("--ref-nu", type=float, default=None)
    c.add_argument("--runs", default="", help="comma list of cold,warm,cold_same (default all)")
    c.add_argument("--finish-storage", default=None, choices=["fp32", "fp64", "fp16s", "fp16c"],
                   help="continue every run from its state at --tol in this storage")
    c.add_argument("--finish-tol", type=float, default=1e-8)
    c.add_argument("--symmetrize", action="store_true",
                   help="average the prediction over the side-heated cell's symmetries")
    a = ap.parse_args()
    say = lambda s: print(s, flush=True)  # noqa: E731
    if a.cmd == "train":
        from .sweep import run_sweep
        fields, info = run_sweep(K=a.K, M=a.M, max_steps=a.sweep_steps, log=say)
        say(f"# sweep: {info['converged']} converged, {info['diverged']} diverged, "
            f"{info['wall_s']:.1f} s")
        net, hist = train(fields, info["cavities"], a.iters, a.batch, a.lr, a.holdout, log=say)
        params = L.lws_net_get_params(net)
        if a.out:
            np.savez(a.out, params=params, M=a.M, ch=np.array(CH),
                     holdout=np.array([[c["Ra"], c["Pr"]] for c in info["cavities"][-a.holdout:]]))
        print(json.dumps({"sweep_converged": info["converged"], "sweep_wall_s": info["wall_s"],
                          "history": hist, "params": int(params.size)}), flush=True)
    else:
        d = np.load(a.params)
        net = L.lws_net_create(int(d["M"]), 1, tuple(int(x) for x in d["ch"]))
        L.lws_net_set_params(net, d["params"])
        r = compare(net, a.N, a.Ra, a.Pr, a.storage, a.check, a.tol, a.max_steps, a.probe,
                    ref_nu=a.ref_nu, cold_storage=a.cold_storage,
                    runs=[x for x in a.runs.split(",") if x] or None, symmetrize=a.symmetrize,
                    finish_storage=a.finish_storage, finish_tol=a.finish_tol, decay=a.decay, log=say)
        print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()


def _track(h, check, tol, max_steps, nu_every, log, tag):
    """Advance h in chunks of nu_every steps with the steady-state check every
    `check` steps until max |dT| < tol or max_steps; after every chunk record
    (step, Nu_hot, Nu_cold, seconds since the start).  Returns the run record."""
    steps, r, hist, track = 0, float("inf"), [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while steps < max_steps and not r < tol:
        n = min(nu_every, max_steps - steps)
        k, r, hh = B.lbm_run_to_steady(h, check, tol, n, history_len=n // check + 1)
        steps += k
        hist += hh
        o = _nu(h)
        track.append((steps, o["Nu_hot"], o["Nu_cold"], time.perf_counter() - t0))
    wall = time.perf_counter() - t0
    log(f"# {tag}: {steps} steps, max_dT {r:.3e}, {wall:.2f} s")
    return {"steps": steps, "max_dT": r, "converged": r < tol, "wall_s": wall, "history": hist,
            "nu_track": track}


def _time_at(track, step):
    for row in track:
        if row[0] == step:
            return row[3]
    return None


def steady_benchmark(N=65, Ra=1e6, Pr=0.71, sweep_K=64, sweep_steps=200_000, iters=1500, holdout=8,
                     check=1000, nu_every=1000, probe=20_000, decay=10.0, ref_tol=1e-9,
                     max_steps=800_000, seed=synth.SEED0 + 1, log=print):
    """Steps and seconds to a steady side-heated cell, the plain method against
    the learned warm start in 16-bit storage, measured end to end on this GPU:

    1. the network is trained here: the batched 64-cavity sweep (run_sweep)
       gives its training fields, then Adam (train);
    2. an FP64-storage run from rest to max |dT| < ref_tol gives the reference
       Nu (mean of the hot- and cold-wall link-flux Nusselt numbers);
    3. three runs of the same cell, each to the max |dT| its storage can reach
       (FP32: 2e-6, FP16C: 1e-4; their rounding floors lie near 1e-6 and
       1e-4): the plain method (FP32 from rest + seeded noise), FP16C from
       rest, and FP16C from the network's prediction averaged over the cell's
       symmetries.  The warm run passes or fails the causal fall-back rule at
       the probe; failing, its strategy is charged the probe plus the FP16C
       run from rest.

    For each run: steps and seconds until the mean wall Nu enters and stays
    within +-0.5% of the reference, and until the residual criterion; the
    final Nu against the reference."""
    from .sweep import run_sweep
    out = {"workload": f"side-heated {N}^3, Ra {Ra:g}, Pr {Pr:g}, Ma 0.1, rest + seeded noise",
           "check": check, "nu_every": nu_every}
    t0 = time.perf_counter()
    fields, info = run_sweep(K=sweep_K, M=M_DEFAULT, max_steps=sweep_steps, log=lambda s: None)
    t_sweep = time.perf_counter() - t0
    net, hist = train(fields, info["cavities"], iters=iters, holdout=holdout, log=lambda s: None)
    del fields
    torch.cuda.empty_cache()
    out["training"] = {"sweep_cavities": sweep_K, "sweep_steps": sweep_steps,
                       "sweep_converged": info["converged"], "sweep_s": round(t_sweep, 2),
                       "train_iters": iters, "train_s": round(hist[-1]["s"], 2),
                       "train_loss": hist[-1]["train_loss"], "holdout_loss": hist[-1]["holdout_loss"]}
    log(f"# steady leg: sweep {t_sweep:.1f} s, training {hist[-1]['s']:.1f} s")
    rest = torch.from_numpy(synth.rest_with_noise(N, seed).reshape(-1)).cuda()
    h = B.lbm_create(N, Ra, Pr, "side_heated", "fp64")
    B.lbm_set_fields(h, rest)
    ref = _track(h, check, ref_tol, 3 * max_steps, 10 * check, log, "fp64 reference")
    nu_ref = 0.5 * (ref["nu_track"][-1][1] + ref["nu_track"][-1][2])
    B.lbm_destroy(h)
    out["reference"] = {"storage": "fp64", "tol_max_dT": ref_tol, "steps": ref["steps"],
                        "converged": ref["converged"], "Nu": nu_ref}
    plan = [("plain_fp32_rest", "fp32", False, 2e-6), ("fp16c_rest", "fp16c", False, 1e-4),
            ("fp16c_warm_symmetrized", "fp16c", True, 1e-4)]
    runs = {}
    for tag, st, warm, tol in plan:
        h = B.lbm_create(N, Ra, Pr, "side_heated", st)
        B.lbm_set_fields(h, predict_fields(net, N, Ra, Pr, symmetrize=True) if warm else rest)
        r = _track(h, check, tol, max_steps, nu_every, log, tag)
        B.lbm_destroy(h)
        s_nu = steps_to_nu([row[:3] for row in r["nu_track"]], nu_ref, wall="mean")
        last = r["nu_track"][-1]
        runs[tag] = {"storage": st, "start": "network (symmetrized)" if warm else "rest + noise",
                     "steps_to_nu_0.5pct": s_nu, "seconds_to_nu_0.5pct": _time_at(r["nu_track"], s_nu),
                     "tol_max_dT": tol, "steps_to_tol": r["steps"] if r["converged"] else None,
                     "seconds_to_tol": round(r["wall_s"], 3) if r["converged"] else None,
                     "final_max_dT": r["max_dT"],
                     "final_Nu_rel_to_ref": (0.5 * (last[1] + last[2]) - nu_ref) / nu_ref,
                     "residual_at_first_check": r["history"][0] if r["history"] else None,
                     "residual_at_probe": (r["history"][probe // check - 1]
                                           if len(r["history"]) >= probe // check else None)}
        if warm:
            keep = keep_warm_start(r["history"], check, probe, decay)
            runs[tag]["kept_by_fallback_rule"] = keep
            if not keep:   # the strategy pays the probe and the FP16C start from rest
                base = runs["fp16c_rest"]
                pst = probe
                pwall = next((row[3] for row in r["nu_track"] if row[0] >= probe), r["wall_s"])
                for k in ("steps_to_nu_0.5pct", "steps_to_tol"):
                    runs[tag][k] = None if base[k] is None else base[k] + pst
                for k in ("seconds_to_nu_0.5pct", "seconds_to_tol"):
                    runs[tag][k] = None if base[k] is None else base[k] + pwall
    out["runs"] = runs
    plain, best = runs["plain_fp32_rest"], runs["fp16c_warm_symmetrized"]
    if plain["steps_to_nu_0.5pct"] and best["steps_to_nu_0.5pct"]:
        out["gain_steps_to_nu"] = plain["steps_to_nu_0.5pct"] / best["steps_to_nu_0.5pct"]
        out["gain_seconds_to_nu"] = plain["seconds_to_nu_0.5pct"] / best["seconds_to_nu_0.5pct"]
    out["leg_s"] = round(time.perf_counter() - t0, 1)
    return out
