"""What the trained warm-start network gains over a start from rest, end to
end on the GPU at a size that runs in seconds: twelve 17^3 side-heated
cavities (Pr 0.71, six with Ra log-spaced on [1e4, 2e4] and six on
[5e4, 1e5]) are advanced to steady state in one batch, their fields
resampled to 17^3 train the network, and a cavity inside the held-out band
(Ra 3e4, 1.5 to 1.7 times away from the nearest training cavities) is run to
the same steady-state criterion from rest and from the network's prediction,
plain and averaged over the cell's symmetries, and once more in two
precision stages (FP16C, then FP64) against an FP64 start from rest.  The
warm start must pass the fall-back rule on its own residual, and its gain is
counted as the strategy's (the probe would be charged had it fallen back)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1903_08882_amd import binding as B  # noqa: E402
from paper_1903_08882_amd import lws as L  # noqa: E402
from paper_1903_08882_amd import synth  # noqa: E402
from paper_1903_08882_amd import warmstart as WS  # noqa: E402


def say(*a):
    print(*a, flush=True)


def steady_fields(N, M, Ras, Pr, tol):
    K = len(Ras)
    b = B.lbm_batch_create([N] * K, Ras, [Pr] * K, [0] * K, "fp32")
    for k in range(K):
        f = torch.from_numpy(synth.rest_with_noise(N, synth.SEED0 + 50 + k).reshape(-1)).cuda()
        B.lbm_set_fields(B.lbm_batch_cavity(b, k), f)
    steps, res = B.lbm_batch_run_to_steady(b, 500, tol, 200_000)
    assert all(r < tol for r in res), res
    fields = torch.empty((K, 4, M, M, M), dtype=torch.float32, device="cuda")
    for k in range(K):
        B.lbm_resample_fields(B.lbm_batch_cavity(b, k), M, out=fields[k].view(-1))
    torch.cuda.synchronize()
    return fields, max(steps)


def test_warm_start_reaches_steady_state_in_fewer_steps():
    N = M = 17
    Pr = 0.71
    Ras = list(10 ** np.linspace(4, np.log10(2e4), 6)) + list(10 ** np.linspace(np.log10(5e4), 5, 6))
    fields, sweep_steps = steady_fields(N, M, Ras, Pr, 2e-6)
    say(f"[warm start] training data: 12 cavities steady after <= {sweep_steps} steps")
    cav = [{"N": N, "Ra": r, "Pr": Pr} for r in Ras]
    net, hist = WS.train(fields, cav, iters=400, batch=6, lr=3e-3, holdout=0, ch=(16, 16, 16),
                         log=lambda s: None)
    say(f"[warm start] loss {hist[0]['train_loss']:.3e} -> {hist[-1]['train_loss']:.3e}")
    assert hist[-1]["train_loss"] < 0.05 * hist[0]["train_loss"]
    for sym in (False, True):
        r = WS.compare(net, N, 3e4, Pr, storage="fp32", check=500, tol=2e-6, max_steps=200_000, probe=2000,
                       symmetrize=sym, log=lambda s: None)
        say(f"[warm start] symmetrize={sym}: cold {r['cold']['steps']} steps, warm {r['warm']['steps']} steps, "
            f"strategy {r['strategy_steps']} (kept {r['kept_warm_start']}), "
            f"Nu cold {r['cold']['Nu']['Nu_hot']:.5f} warm {r['warm']['Nu']['Nu_hot']:.5f}")
        say("[warm start] residuals of the first checks: cold "
            + " ".join(f"{v:.2e}" for v in r["cold_history_head"][:10]) + " | warm "
            + " ".join(f"{v:.2e}" for v in r["warm_history_head"][:10]))
        assert r["cold"]["converged"] and r["warm"]["converged"]
        assert r["kept_warm_start"]
        assert r["strategy_steps"] <= 0.75 * r["cold"]["steps"]
        assert abs(r["Nu_rel_diff_warm_vs_cold"]) < 5e-3
    # staged precision: a 16-bit stage to 1e-4, then FP64 to 1e-9, against an
    # FP64 cold start to the same criterion: both reach the same steady state
    r = WS.compare(net, N, 3e4, Pr, storage="fp16c", cold_storage="fp64", check=500, tol=1e-4,
                   max_steps=200_000, probe=2000, symmetrize=True, finish_storage="fp64", finish_tol=1e-9,
                   runs=["cold", "warm"], log=lambda s: None)
    say(f"[warm start] staged fp16c -> fp64: cold {r['cold']['steps']} steps, warm {r['warm']['steps']} "
        f"(first stage {r['warm']['stage1']['steps']})")
    assert r["cold"]["converged"] and r["warm"]["converged"]
    assert r["warm"]["stage1"]["converged"] and r["warm"]["storage"] == "fp16c"
    assert abs(r["Nu_rel_diff_warm_vs_cold"]) < 1e-6
