"""Throughput of the coupled D3Q19-MRT / D3Q7-MRT thermal LB step on one GPU.

Workload (default): side-heated cubic cell, 257^3 nodes, Ra = 1e7, Pr = 0.71,
Mach 0.1 (U = 0.1/sqrt 3), FP32 populations, fluid at rest with seeded +-1e-3
temperature noise.  One "step" is one coupled time step of the whole hot path
as the steady-state driver runs it: the fused stream-collide kernel every
step, the observable reductions accumulated into the FP64 time averages every
100 steps, and the steady-state residual every 1000 steps.  Inputs are
resident in HBM before the timed region starts.

Prints one JSON line.  Value = million lattice updates per second (both
lattices at one node = one update).  The roofline entry uses the step
kernel's mean duration from HIP events around each launch in the timed region
and its algorithmic traffic: 26 populations read and written per node.

The second half of the metric, steps to steady state against the plain
method, is the "steps_to_steady" record (outside the timed region): the
side-heated 65^3 cell at Ra 1e6 from rest in FP32 (the plain method) against
FP16C storage started from the warm-start network, which the leg trains on
this GPU first (warmstart.steady_benchmark).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
METRIC = "coupled-lattice MLUPS & % HBM roofline; steps-to-steady vs plain at Nu ±0.5%"
# bytes of one node's 26 populations in HBM (FP16 storage keeps the seven
# thermal populations in FP32); a step reads and writes each once
NODE_BYTES = {"fp64": 26 * 8, "fp32": 26 * 4, "fp16s": 19 * 2 + 7 * 4, "fp16c": 19 * 2 + 7 * 4}
DTYPE = {"fp64": "f64", "fp32": "f32", "fp16s": "f16 storage / f32 compute",
         "fp16c": "custom 16-bit storage / f32 compute"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--N", type=int, default=257)
    ap.add_argument("--Ra", type=float, default=1e7)
    ap.add_argument("--Pr", type=float, default=0.71)
    ap.add_argument("--cell", default="side_heated", choices=["side_heated", "rayleigh_benard"])
    ap.add_argument("--storage", default="fp32", choices=["fp32", "fp64", "fp16s", "fp16c"])
    ap.add_argument("--sample-every", type=int, default=100)
    ap.add_argument("--residual-every", type=int, default=1000)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--waves", type=int, nargs=2, default=(0, 0), metavar=("EVEN", "ODD"),
                    help="occupancy caps of the step kernel (0 = library default, -1 = none)")
    ap.add_argument("--cpu-steps", type=int, default=30,
                    help="oracle steps of the CPU baseline sample (0 = skip)")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="measured HBM bytes per step-kernel launch, if recorded")
    ap.add_argument("--copy-mib", type=int, default=1024,
                    help="size of the device-copy reference measured after the run (0 = skip)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--steady-leg", type=int, default=1,
                    help="1: also measure steps and seconds to steady state, plain FP32 from rest "
                         "against FP16C from the network trained here (0 = skip)")
    ap.add_argument("--leg-N", type=int, default=65)
    ap.add_argument("--leg-Ra", type=float, default=1e6)
    ap.add_argument("--leg-sweep-steps", type=int, default=200_000)
    return ap.parse_args()


def kernel_source_hash():
    """Hash of the kernel source: recorded traffic is valid for this source only."""
    import hashlib
    h = hashlib.sha1()
    for f in ("kernels.hip", "lbm_internal.h"):
        with open(os.path.join(ROOT, "paper_1903_08882_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def cpu_baseline(a):
    """The FP64 oracle, as it stands, on the host cores: a bounded sample of
    the same workload (same N, same initial state, a few steps)."""
    import oracle
    from paper_1903_08882_amd import synth

    o = oracle.Oracle(a.N, a.Ra, a.Pr, oracle.SIDE_HEATED if a.cell == "side_heated"
                      else oracle.RAYLEIGH_BENARD)
    o.init_fields(synth.rest_with_noise(a.N))
    o.step(1)  # first touch of both arrays outside the timing
    t0 = time.perf_counter()
    o.step(a.cpu_steps)
    dt = time.perf_counter() - t0
    return {"value": round(a.N ** 3 * a.cpu_steps / dt / 1e6, 3), "unit": "MLUPS",
            "cores": oracle.threads(), "kind": "oracle",
            "sample": f"{a.cpu_steps} FP64 oracle steps of the same {a.N}^3 workload "
                      f"({dt:.1f} s)"}


def main():
    a = parse()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the method is built and measured on a single "
              "MI355X here (multi-GPU slab decomposition is a design, not built).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1903_08882_amd import binding as B
    from paper_1903_08882_amd import synth

    torch.cuda.set_device(0)
    N = a.N
    opts = B.lbm_default_opts(sample_every=a.sample_every, block=a.block, waves_even=a.waves[0],
                              waves_odd=a.waves[1])
    h = B.lbm_create(N, a.Ra, a.Pr, a.cell, a.storage, opts)
    fields = torch.from_numpy(synth.rest_with_noise(N).reshape(-1)).cuda()
    B.lbm_set_fields(h, fields)
    del fields
    stream = torch.cuda.current_stream()

    def run(steps):
        done, last = 0, None
        while done < steps:
            k = min(a.residual_every - (B.lbm_time(h) % a.residual_every), steps - done)
            B.lbm_step(h, k, stream)
            done += k
            if B.lbm_time(h) % a.residual_every == 0:
                last = B.lbm_residual(h, stream)
        return last

    run(a.warmup)
    torch.cuda.synchronize()
    B.lbm_profile(h, True)
    B.lbm_profile_read(h)
    t0 = time.perf_counter()
    res = run(a.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kernel_ms, kernels = B.lbm_profile_read(h)
    B.lbm_profile(h, False)
    Nu, Re, eps_u, eps_T = B.lbm_observables(h, stream)

    V = N ** 3
    mlups = V * a.steps / elapsed / 1e6
    bytes_step = 2 * NODE_BYTES[a.storage] * V
    avg_kernel_s = kernel_ms / 1e3 / max(kernels, 1)
    achieved = bytes_step / avg_kernel_s / 1e9
    traffic = None
    if os.path.exists(a.traffic_json):
        tj = json.load(open(a.traffic_json))
        rec = tj.get(f"{a.cell}:{N}:{a.storage}")
        if rec and rec.get("kernel_source") == kernel_source_hash():
            traffic = rec["bytes_per_launch"]
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(elapsed / a.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[a.storage],
        "data": "synthetic",
        "config": {"workload": f"{a.cell.replace('_', '-')} cubic cell {N}^3, Ra={a.Ra:g}, "
                               f"Pr={a.Pr:g}, Ma=0.1, D3Q19-MRT + D3Q7-MRT, "
                               f"{a.storage.upper()} populations, rest + seeded T noise",
                   "N": N, "Ra": a.Ra, "Pr": a.Pr, "cell": a.cell, "storage": a.storage,
                   "sample_every": a.sample_every, "residual_every": a.residual_every,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "kernel": f"k_step ({a.storage}, {kernels} launches, "
                               f"mean {avg_kernel_s * 1e6:.1f} us, {bytes_step / V:.0f} B/node)"},
        "whole_step_hbm_frac": round(bytes_step / (elapsed / a.steps) / 1e9 / HBM_PEAK_GBS, 4),
        "observables": {"Nu": Nu, "Re": Re, "eps_u": eps_u, "eps_T": eps_T,
                        "residual_max_dT": res[0] if res else None,
                        "residual_interval": a.residual_every},
    }
    del h
    torch.cuda.empty_cache()
    if a.copy_mib > 0:
        # the same GPU's practical HBM ceiling: the library's reference copy
        # (16-byte streaming loads and stores), timed with HIP events
        src = torch.ones(a.copy_mib * (1 << 18), dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            B.lbm_device_copy(dst, src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            B.lbm_device_copy(dst, src)
        e1.record()
        torch.cuda.synchronize()
        copy_gbs = 2 * src.numel() * 4 * 20 / (e0.elapsed_time(e1) / 1e3) / 1e9
        out["device_copy"] = {"GB/s": round(copy_gbs, 1), "bytes": 2 * src.numel() * 4,
                              "kernel": "lbm_device_copy (16-byte streaming loads and stores)",
                              "step_kernel_frac_of_copy": round(achieved / copy_gbs, 4)}
        del src, dst
    if a.calibrate_copy:
        n = a.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = 4 * n
        del src, dst
    if a.steady_leg:
        from paper_1903_08882_amd import warmstart
        out["steps_to_steady"] = warmstart.steady_benchmark(
            N=a.leg_N, Ra=a.leg_Ra, sweep_steps=a.leg_sweep_steps,
            log=lambda m: print(m, file=sys.stderr, flush=True))
    out["cpu_baseline"] = cpu_baseline(a) if a.cpu_steps > 0 else None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
