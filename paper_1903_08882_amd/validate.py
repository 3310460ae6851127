"""Side-heated cavity to steady state on the GPU, compared with the paper's
benchmark values (Sec. 3, Tables 1 and 2).

    python -m paper_1903_08882_amd.validate --N 129 --Ra 1e6

Runs the C-ABI steady-state driver (max |dT| over `--check` steps below
`--tol`) from rest with seeded noise (or, with --init-from N0, from the
steady fields of an N0^3 run resampled onto the grid), then reports the
plane-averaged Nusselt profile across the cell (Sec. 3, Fig. 4), the hot- and cold-wall
Nusselt numbers (overall and mid-plane line; link flux and one-sided
difference), the mid-plane centreline velocity maxima with their positions,
the kinetic energy E, and the paper's values for the same grid and Ra.  The
paper's hot and cold walls are y = 0 and y = 1; here they are x = 0 and x = 1,
so its v_max (location z) is our u_max (location z) and its w_max (location y)
is our w_max (location x).
"""
import argparse
import json
import time

import torch

from . import binding as B
from . import synth

# Sec. 3, Table 1 (v_max, z, w_max, y, E x 1e3) and Table 2 (Nu_mean and
# Nu_overall at the hot wall y = 0 and the cold wall y = 1), "Present" rows.
PAPER = {
    (81, 1e6): dict(v_max=0.08056, z=0.8580, w_max=0.25437, y=0.0432, E=3.3346e-3,
                    Nu_mean_hot=8.99850, Nu_mean_cold=8.99333, Nu_hot=8.75450, Nu_cold=8.75405),
    (129, 1e6): dict(v_max=0.08091, z=0.8566, w_max=0.25753, y=0.0349, E=3.3280e-3,
                     Nu_mean_hot=8.91688, Nu_mean_cold=8.91467, Nu_hot=8.67775, Nu_cold=8.67746),
    (161, 1e6): dict(v_max=0.08099, z=0.8540, w_max=0.25729, y=0.0404, E=3.3265e-3,
                     Nu_mean_hot=8.89886, Nu_mean_cold=8.89744, Nu_hot=8.66075, Nu_cold=8.66060),
    (257, 1e6): dict(v_max=0.08107, z=0.8541, w_max=0.25836, y=0.0370, E=3.3248e-3,
                     Nu_mean_hot=8.88054, Nu_mean_cold=8.87994, Nu_hot=8.64345, Nu_cold=8.64342),
    (81, 1e7): dict(v_max=0.05410, z=0.8951, w_max=0.25865, y=0.0185, E=1.8418e-3,
                    Nu_mean_hot=17.26877, Nu_mean_cold=17.31377, Nu_hot=17.03864, Nu_cold=17.09483),
    (129, 1e7): dict(v_max=0.05671, z=0.8798, w_max=0.26054, y=0.0194, E=1.8365e-3,
                     Nu_mean_hot=16.85522, Nu_mean_cold=16.85465, Nu_hot=16.64342, Nu_cold=16.64642),
    (161, 1e7): dict(v_max=0.05730, z=0.8789, w_max=0.26184, y=0.0217, E=1.8345e-3,
                     Nu_mean_hot=16.73787, Nu_mean_cold=16.73588, Nu_hot=16.52963, Nu_cold=16.52950),
    (257, 1e7): dict(v_max=0.05789, z=0.8774, w_max=0.26181, y=0.0214, E=1.8322e-3,
                     Nu_mean_hot=16.60871, Nu_mean_cold=16.60782, Nu_hot=16.40322, Nu_cold=16.40285),
}


# Sec. 3, Table 3: rms density fluctuation and rms velocity divergence.
TABLE3 = {
    (81, 1e6): dict(rms_drho=1.4793e-3, rms_div=1.994e-2), (129, 1e6): dict(rms_drho=1.4794e-3, rms_div=8.779e-3),
    (161, 1e6): dict(rms_drho=1.4794e-3, rms_div=5.722e-3), (257, 1e6): dict(rms_drho=1.4795e-3, rms_div=2.228e-3),
    (81, 1e7): dict(rms_drho=1.4770e-3, rms_div=4.183e-2), (129, 1e7): dict(rms_drho=1.4788e-3, rms_div=2.295e-2),
    (161, 1e7): dict(rms_drho=1.4791e-3, rms_div=1.617e-2), (257, 1e7): dict(rms_drho=1.4795e-3, rms_div=7.132e-3),
}


def richardson(ns, fs):
    """Order p and extrapolated value f_inf of f(h) = f_inf + C h^p, h = 1/N,
    through three grids N1 < N2 < N3 (ratios need not be equal): p solves
    (f1 - f2) / (f2 - f3) = (h1^p - h2^p) / (h2^p - h3^p) (by bisection on
    [0.05, 20]), then C = (f1 - f2) / (h1^p - h2^p) and f_inf = f3 - C h3^p.
    Returns (p, f_inf); (nan, nan) when the three values do not converge
    monotonically."""
    (n1, n2, n3), (f1, f2, f3) = ns, fs
    h1, h2, h3 = 1.0 / n1, 1.0 / n2, 1.0 / n3
    if (f1 - f2) * (f2 - f3) <= 0.0:
        return float("nan"), float("nan")
    target = (f1 - f2) / (f2 - f3)

    def g(p):
        return (h1 ** p - h2 ** p) / (h2 ** p - h3 ** p) - target

    lo, hi = 0.05, 20.0
    if g(lo) * g(hi) > 0.0:
        return float("nan"), float("nan")
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if g(lo) * g(mid) <= 0.0:
            hi = mid
        else:
            lo = mid
    p = 0.5 * (lo + hi)
    c = (f1 - f2) / (h1 ** p - h2 ** p)
    return p, f3 - c * h3 ** p


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--N", type=int, default=129)
    ap.add_argument("--Ra", type=float, default=1e6)
    ap.add_argument("--Pr", type=float, default=0.71)
    ap.add_argument("--storage", default="fp32", choices=["fp32", "fp64", "fp16s", "fp16c"])
    ap.add_argument("--check", type=int, default=1000)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--max-steps", type=int, default=2_000_000)
    ap.add_argument("--start-storage", default=None, choices=["fp32", "fp64", "fp16s", "fp16c"],
                    help="reach --start-tol in this storage first, then carry the populations over")
    ap.add_argument("--start-tol", type=float, default=1e-5)
    ap.add_argument("--start-max-steps", type=int, default=2_000_000)
    ap.add_argument("--T0", type=float, default=0.0,
                    help="reference temperature of the buoyancy (walls at +-0.5)")
    ap.add_argument("--init-from", type=int, default=0, metavar="N0",
                    help="start from the steady fields of an N0^3 FP32 run (to --init-tol), "
                         "resampled trilinearly onto N^3, instead of from rest")
    ap.add_argument("--init-tol", type=float, default=2e-6)
    a = ap.parse_args()

    t0 = time.perf_counter()
    start_steps = 0
    init = torch.from_numpy(synth.rest_with_noise(a.N).reshape(-1)).cuda()
    coarse = None
    if a.init_from:
        hc = B.lbm_create(a.init_from, a.Ra, a.Pr, "side_heated", "fp32", B.lbm_default_opts(T0=a.T0))
        B.lbm_set_fields(hc, torch.from_numpy(synth.rest_with_noise(a.init_from).reshape(-1)).cuda())
        ks, rc = 0, float("inf")
        while ks < a.start_max_steps and not rc < a.init_tol:
            k, rc, _ = B.lbm_run_to_steady(hc, a.check, a.init_tol, min(100 * a.check, a.start_max_steps - ks))
            ks += k
            print(f"# {a.init_from}^3 fp32 step {ks}  max_dT {rc:.3e}  {time.perf_counter() - t0:.1f} s", flush=True)
        f32 = torch.empty(4 * a.N ** 3, dtype=torch.float32, device="cuda")
        B.lbm_resample_fields(hc, a.N, out=f32)
        init = f32.double()
        del f32
        B.lbm_destroy(hc)
        coarse = {"N": a.init_from, "steps": ks, "max_dT": rc}
    if a.start_storage:
        h0 = B.lbm_create(a.N, a.Ra, a.Pr, "side_heated", a.start_storage, B.lbm_default_opts(T0=a.T0))
        B.lbm_set_fields(h0, init)
        r0 = float("inf")
        while start_steps < a.start_max_steps and not r0 < a.start_tol:
            k, r0, _ = B.lbm_run_to_steady(h0, a.check, a.start_tol,
                                           min(100 * a.check, a.start_max_steps - start_steps))
            start_steps += k
            print(f"# {a.start_storage} step {start_steps}  max_dT {r0:.3e}  {time.perf_counter() - t0:.1f} s",
                  flush=True)
        pop = B.lbm_get_populations(h0)
        B.lbm_destroy(h0)
        h = B.lbm_create(a.N, a.Ra, a.Pr, "side_heated", a.storage, B.lbm_default_opts(T0=a.T0))
        B.lbm_set_populations(h, pop)
        del pop
    else:
        h = B.lbm_create(a.N, a.Ra, a.Pr, "side_heated", a.storage, B.lbm_default_opts(T0=a.T0))
        B.lbm_set_fields(h, init)
    del init
    steps, r, hist = 0, float("inf"), []
    chunk = 100 * a.check                      # report progress every 100 checks
    while steps < a.max_steps and not r < a.tol:
        k, r, hh = B.lbm_run_to_steady(h, a.check, a.tol, min(chunk, a.max_steps - steps),
                                       history_len=100)
        steps += k
        hist += hh
        print(f"# step {steps}  max_dT {r:.3e}  {time.perf_counter() - t0:.1f} s", flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    nd = B.lbm_nondimensional(B.lbm_get_params(h), B.lbm_observables_raw(h))
    pk = B.lbm_centerline_peaks(h)
    prof = B.lbm_nusselt_profile(h)
    nu_w = 0.5 * (nd["Nu_hot"] + nd["Nu_cold"])
    out = {"N": a.N, "Ra": a.Ra, "Pr": a.Pr, "storage": a.storage, "steps": steps,
           "start_storage": a.start_storage, "start_steps": start_steps,
           "max_dT": r, "converged": r < a.tol, "wall_s": round(wall, 2),
           "MLUPS": round(a.N ** 3 * (steps + start_steps) / wall / 1e6, 1),
           "Nu_hot": nd["Nu_hot"], "Nu_cold": nd["Nu_cold"], "Nu_mean_hot": nd["Nu_hot_mid"],
           "Nu_mean_cold": nd["Nu_cold_mid"], "Nu_hot_fd": nd["Nu_hot_fd"],
           "Nu_cold_fd": nd["Nu_cold_fd"], "Nu_mean_hot_fd": nd["Nu_hot_mid_fd"],
           "v_max": pk["u_max"], "z": pk["u_max_z"], "w_max": pk["w_max"], "y": pk["w_max_x"],
           "E": pk["E"], "rms_drho": nd["rms_drho"], "rms_div": nd["rms_div"], "T0": a.T0,
           "nusselt_profile": {"min_rel": min(prof) / nu_w - 1.0, "max_rel": max(prof) / nu_w - 1.0,
                               "mean_rel": sum(prof) / len(prof) / nu_w - 1.0,
                               "every_8th": prof[::8]},
           "coarse_start": coarse,
           "residual_every_10_checks": hist[::10]}
    ref = PAPER.get((a.N, a.Ra))
    if ref and abs(a.Pr - 0.71) < 1e-12:
        ref = dict(ref, **TABLE3.get((a.N, a.Ra), {}))
        out["paper"] = ref
        out["rel_diff"] = {k: (out[k] - v) / v for k, v in ref.items()}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
