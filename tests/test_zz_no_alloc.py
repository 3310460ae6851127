"""The allocation-free weight gradient (lws_conv3d_backward_weight_noalloc,
for callers that cannot allocate device memory) against the entry point with
a caller's workspace (lws_conv3d_backward_weight), through the C ABI, on two
calls in a row, the second smaller than the first: both within the FP32
accumulation bar of the FP64 reference (|dw - ref| <= 1e-5 sum |terms|, the
bar of the convolution parity tests), and equal bit for bit where both use
the same voxel chunks.  The first call (64 -> 64 channels over 2 x 45^3
voxels) needs more partial tiles than the 64 MiB scratch array holds with
the usual chunking, so the allocation-free call coarsens its chunks; the
second (16 -> 8 over 9^3) uses the usual chunking and must leave nothing of
the first call's partials in its result."""
import numpy as np
import pytest

from oracle import wsnet as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1903_08882_amd import lws as L  # noqa: E402
from paper_1903_08882_amd import synth  # noqa: E402


def say(*a):
    print(*a, flush=True)


def bits(a):
    f = W.bf16_round(a).astype(np.float32)
    u = (f.view(np.uint32) >> 16).astype(np.uint16)
    return torch.from_numpy(u.view(np.int16).reshape(-1).copy()).cuda()


def rand(shape, seed, stream):
    return synth.uniform(seed, stream, int(np.prod(shape))).reshape(shape)


def test_weight_gradient_without_allocation_matches_the_workspace_entry_point():
    for k, (B, D, H, Wd, ci, co, same_chunks) in enumerate([(2, 45, 45, 45, 64, 64, False),
                                                            (1, 9, 9, 9, 16, 8, True)]):
        say(f"[no-alloc wgrad] call {k + 1}: B={B} grid {D}x{H}x{Wd} cin={ci} cout={co}")
        X = W.bf16_round(rand((B, D, H, Wd, ci), synth.SEED0 + 300 + k, 0))
        G = W.bf16_round(rand((B, D, H, Wd, co), synth.SEED0 + 300 + k, 1))
        xb, gb = bits(X), bits(G)
        grid = (B, D, H, Wd)
        ws = L.lws_conv3d_backward_weight(xb, 0, ci, gb, co, grid).cpu().numpy()
        out = torch.full((27 * ci * co,), float("nan"), dtype=torch.float32, device="cuda")
        na = L.lws_conv3d_backward_weight_noalloc(xb, 0, ci, gb, co, grid, out).cpu().numpy()
        torch.cuda.synchronize()
        ref = W.conv3d_bwd_weight(X, G).reshape(-1)
        bound = 1e-5 * W.conv3d_bwd_weight(np.abs(X), np.abs(G)).reshape(-1) + 1e-30
        for name, dw in (("workspace", ws), ("no-alloc", na)):
            worst = np.max(np.abs(dw - ref) / bound)
            say(f"[no-alloc wgrad] call {k + 1} {name}: worst error / bar {worst:.3g}")
            assert np.all(np.abs(dw - ref) <= bound), name
        if same_chunks:
            assert np.array_equal(na, ws)
        else:
            assert np.max(np.abs(na - ws) / bound) <= 2.0
