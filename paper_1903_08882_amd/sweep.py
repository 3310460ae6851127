"""Batched sweep: many side-heated cavities of uneven size advanced together to
steady state in one batch (one kernel launch per step for all of them), then
resampled onto a common grid.

    python -m paper_1903_08882_amd.sweep --K 64 --M 65

Cavities: N uniform over {33, 49, 65}, Ra log-uniform over [1e4, 1e7], Pr over
{0.71, 7}, fluid at rest with seeded noise (``synth.sweep_cavities``).  The
block size of the batched launch is autotuned first.  Each cavity retires when
its max |dT| over `--check` steps falls below `--tol` (or diverges); the
steady fields (u, v, w, T) are resampled trilinearly onto M^3 nodes (FP32).
Prints progress lines and one JSON summary (timing of the all-active batched
step in MLUPS and as a fraction of HBM peak).
"""
import argparse
import json
import time

import torch

from . import binding as B
from . import synth

HBM_PEAK_GBS = 8000.0
NODE_BYTES = {"fp64": 26 * 8, "fp32": 26 * 4, "fp16s": 19 * 2 + 7 * 4, "fp16c": 19 * 2 + 7 * 4}


def run_sweep(K=64, storage="fp32", check=1000, tol=2e-6, max_steps=300_000, M=65,
              chunk_checks=20, seed=synth.SEED0 + 3, log=print):
    """Run the sweep; returns (fields [K, 4, M, M, M] float32 on the GPU, info dict)."""
    cs = synth.sweep_cavities(K, seed=seed)
    Ns = [c["N"] for c in cs]
    b = B.lbm_batch_create(Ns, [c["Ra"] for c in cs], [c["Pr"] for c in cs], [0] * K, storage)
    for k, c in enumerate(cs):
        f = torch.from_numpy(synth.rest_with_noise(c["N"], c["seed"]).reshape(-1)).cuda()
        B.lbm_set_fields(B.lbm_batch_cavity(b, k), f)
    blk, _ = B.lbm_batch_autotune(b, 10)
    torch.cuda.synchronize()
    # timed all-active batched steps
    nodes = sum(N ** 3 for N in Ns)
    t0 = time.perf_counter()
    B.lbm_batch_step(b, 200)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 200
    mlups = nodes / dt / 1e6
    frac = nodes * 2 * NODE_BYTES[storage] / dt / 1e9 / HBM_PEAK_GBS
    log(f"# batch of {K} cavities ({nodes / 1e6:.2f} M nodes), block {blk}: "
        f"{dt * 1e3:.3f} ms/step, {mlups:.0f} MLUPS, {frac:.3f} of HBM peak")
    t0 = time.perf_counter()
    done = 200
    steps, res = [200] * K, [float("inf")] * K
    while done < max_steps:
        n = min(chunk_checks * check, max_steps - done)
        steps, res = B.lbm_batch_run_to_steady(b, check, tol, n)
        done += n
        active = sum(1 for r in res if r == r and r >= tol)
        fin = [r for r in res if r == r]
        log(f"# {time.perf_counter() - t0:.1f} s: up to {max(steps)} steps, {active} active, "
            f"max residual {max(fin) if fin else float('nan'):.3e}")
        if active == 0:
            break
    wall = time.perf_counter() - t0
    fields = torch.empty((K, 4, M, M, M), dtype=torch.float32, device="cuda")
    for k in range(K):
        B.lbm_resample_fields(B.lbm_batch_cavity(b, k), M, out=fields[k].view(-1))
    torch.cuda.synchronize()
    info = {"K": K, "storage": storage, "block": blk, "nodes": nodes,
            "batched_ms_per_step": dt * 1e3, "batched_MLUPS": mlups, "batched_hbm_frac": frac,
            "wall_s": wall, "steps": steps, "residual": res,
            "converged": sum(1 for r in res if r == r and r < tol),
            "diverged": sum(1 for r in res if r != r), "cavities": cs}
    return fields, info


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--K", type=int, default=64)
    ap.add_argument("--M", type=int, default=65)
    ap.add_argument("--storage", default="fp32", choices=["fp32", "fp64", "fp16s", "fp16c"])
    ap.add_argument("--check", type=int, default=1000)
    # FP32 storage settles to max |dT| of about 1e-6 per 1000 steps (its
    # rounding floor), so the sweep's default stop is 2e-6
    ap.add_argument("--tol", type=float, default=2e-6)
    ap.add_argument("--max-steps", type=int, default=300_000)
    ap.add_argument("--save", default="", help="torch.save the fields and info to this path")
    a = ap.parse_args()
    fields, info = run_sweep(a.K, a.storage, a.check, a.tol, a.max_steps, a.M,
                             log=lambda s: print(s, flush=True))
    if a.save:
        torch.save({"fields": fields.cpu(), "info": info}, a.save)
    out = {k: v for k, v in info.items() if k not in ("cavities",)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
