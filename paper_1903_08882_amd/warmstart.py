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
state check (max |dT| over `--check` steps) to `--tol`.  After `--probe` steps
the warm run's residual is compared with the cold run's at the same step; if
it is not smaller the prediction is dropped and the cold run's count stands
(fall back).  Reports steps, wall time, the hot-wall Nusselt numbers of both
runs and their relative difference, and the reference value when given.
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
            at_probe = (steps, r)
        o = _nu(h)
        nu.append((steps, o["Nu_hot"], o["Nu_cold"]))
        log(f"# {tag}: step {steps}  max_dT {r:.3e}  Nu_hot {o['Nu_hot']:.4f}  Nu_cold {o['Nu_cold']:.4f}  "
            f"{time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    return {"steps": steps, "max_dT": r, "converged": r < tol, "wall_s": time.perf_counter() - t0,
            "probe": at_probe, "history": hist, "nu_track": nu}


def keep_warm_start(warm_probe, cold_probe):
    """The fallback rule: keep the warm start only if, at the probe step, its
    steady-state residual (max |dT| over one check interval) is below the cold
    start's.  Probes are (step, residual) or None; a residual that is not a
    number (a diverged run) never wins."""
    if warm_probe is None or cold_probe is None:
        return False
    w, c = warm_probe[1], cold_probe[1]
    if not (w == w) or w == float("inf"):
        return False
    return not (c == c) or w < c


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
            finish_storage=None, finish_tol=None, log=print):
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
    # fall back: the warm start is kept only if its residual at the probe beats
    # that of the cold start in the same storage
    base = res.get("cold_same", cold)
    keep = keep_warm_start(warm["probe"], base["probe"])
    chosen = warm if keep else base
    out.update({"cold": {k: v for k, v in cold.items() if k != "history"},
                "warm": {k: v for k, v in warm.items() if k != "history"},
                "kept_warm_start": keep,
                "steps_saved": cold["steps"] - chosen["steps"],
                "speedup_steps": cold["steps"] / max(chosen["steps"], 1),
                "speedup_wall": cold["wall_s"] / max(chosen["wall_s"], 1e-9),
                "Nu_rel_diff_warm_vs_cold": (warm["Nu"]["Nu_hot"] - cold["Nu"]["Nu_hot"]) / cold["Nu"]["Nu_hot"],
                "cold_history_every_10": cold["history"][::10],
                "warm_history_every_10": warm["history"][::10]})
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
                    finish_storage=a.finish_storage, finish_tol=a.finish_tol, log=say)
        print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
