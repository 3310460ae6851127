"""The C ABI from a C program (paper_1903_08882_amd/examples/c_abi_demo.c,
built by build() with gcc against the library and the HIP runtime): the
library allocates its own device memory (dev_buf = NULL) and the program runs
the 33^3 side-heated cell to steady state.  The same run through the Python
binding (torch-owned buffer) must give the same steps and the same
observables bit for bit: the two paths share every kernel and launch."""
import json
import os
import subprocess

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1903_08882_amd import binding as B  # noqa: E402
from paper_1903_08882_amd import build as BUILD  # noqa: E402


def demo_fields(N):
    z, y, x = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    uvwT = np.zeros((4, N, N, N))
    uvwT[3] = 1e-3 * (((7 * x + 13 * y + 29 * z) % 17) - 8) / 8.0
    return uvwT


@pytest.mark.parametrize("storage", ["fp32", "fp16c"])
def test_c_program_matches_python_binding(storage):
    if not os.path.exists(BUILD.DEMO_PATH):
        pytest.fail("the C example is not built (run build())")
    N, Ra = 33, 1e4
    code = B.STORAGES[storage]
    print(f"[c abi] N={N} Ra={Ra} storage={storage}", flush=True)
    r = subprocess.run([BUILD.DEMO_PATH, str(N), repr(Ra), str(code)], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    c = json.loads(r.stdout.strip().splitlines()[-1])
    h = B.lbm_create(N, Ra, 0.71, "side_heated", storage, B.lbm_default_opts(U=0.1))
    B.lbm_set_fields(h, torch.from_numpy(demo_fields(N).reshape(-1)).cuda())
    steps, res, _ = B.lbm_run_to_steady(h, 1000, 1e-6, 200_000)
    Nu, Re, eps_u, eps_T = B.lbm_observables(h)
    print(f"[c abi] C: {c['steps']} steps Nu {c['Nu']:.9f}; Python: {steps} steps Nu {Nu:.9f}", flush=True)
    assert c["steps"] == steps and c["max_dT"] == res
    assert (c["Nu"], c["Re"], c["eps_u"], c["eps_T"]) == (Nu, Re, eps_u, eps_T)
