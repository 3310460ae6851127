"""CPU tests of the HIP library's host side: it loads, exports every symbol
that include/lbm.h declares, and its host-only calls (parameter derivation,
state size, conversion to nondimensional numbers, argument checks) agree with
the oracle.  No GPU call is made."""
import math
import os
import re

import numpy as np
import pytest

import oracle
from conftest import ROOT

torch = pytest.importorskip("torch")
from paper_1903_08882_amd import binding as B  # noqa: E402

HEADER = os.path.join(ROOT, "include", "lbm.h")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^LBM_API[^(]*?\b(lbm_\w+)\(", text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    syms = declared_symbols()
    assert len(syms) >= 20
    lib = B.lib()
    for s in syms:
        assert hasattr(lib, s), s
    # and the binding wraps each of them under the same name
    for s in syms:
        assert hasattr(B, s) or s in ("lbm_last_error", "lbm_strerror", "lbm_batch_last_error"), s


def test_binding_signature_table_covers_header():
    assert set(declared_symbols()) == set(B._SIG)


@pytest.mark.parametrize("cfg", [(33, 1e4, 0.71, 0, 0.1), (129, 1e6, 0.71, 0, None),
                                 (257, 1e7, 0.71, 0, None), (257, 3e6, 7.0, 1, None),
                                 (65, 1e5, 7.0, 1, None)])
def test_derived_parameters_agree_with_oracle(cfg):
    N, Ra, Pr, cell, U = cfg
    opts = B.lbm_default_opts(U=U)
    p = B.lbm_derive_params(N, Ra, Pr, cell, "fp32", opts)
    q = oracle.derive(N, Ra, Pr, cell, p.U)
    for k in ("H", "dT", "nu", "kappa", "gbeta", "tau_f", "s_e", "s_q", "q_k", "q_e", "q_nu",
              "a_T", "wT0", "wT1", "T_hot", "T_cold"):
        assert abs(getattr(p, k) - getattr(q, k)) <= 1e-15 * max(1.0, abs(getattr(q, k))), k
    if U is None:
        assert abs(p.U - 0.1 / math.sqrt(3)) < 1e-16


def test_parameter_errors():
    with pytest.raises(B.LBMError) as e:
        B.lbm_derive_params(2, 1e4, 0.71)
    assert e.value.status == -1
    with pytest.raises(B.LBMError) as e:
        B.lbm_derive_params(33, 1e3, 0.71, opts=B.lbm_default_opts(U=0.1))
    assert e.value.status == -2       # a_T > 1: negative D3Q7 rest weight
    with pytest.raises(B.LBMError):
        B.lbm_derive_params(33, -1.0, 0.71)
    with pytest.raises(B.LBMError):
        B.lbm_derive_params(33, 1e4, float("nan"))
    with pytest.raises(B.LBMError):
        B.lbm_derive_params(33, 1e4, 0.71, cell=7)
    with pytest.raises(B.LBMError):
        B.lbm_derive_params(33, 1e4, 0.71, storage=9)
    with pytest.raises(B.LBMError) as e:
        B.lbm_derive_params(1601, 1e4, 0.71)
    assert e.value.status == -2


def test_state_bytes_cover_populations_and_scratch():
    for N, st, es, nb in [(33, "fp32", 4, 104), (257, "fp32", 4, 104), (257, "fp64", 8, 208),
                          (129, "fp16s", 2, 66), (129, "fp16c", 2, 66)]:
        b = B.lbm_state_bytes(N, st)
        pops = nb * N ** 3
        scratch = (5 + 4) * N ** 3 * 8
        # node blocks pad each z-plane to whole sub-blocks: at most 2x for
        # lattices smaller than one sub-block, at most one sub-block per plane
        sub = 32768 // es * nb
        pad = min(pops, N * sub)
        assert pops + scratch <= b <= pops + pad + scratch + 64 * N * N * 8 + (1 << 20)


@pytest.mark.parametrize("cell", [0, 1])
def test_nondimensional_conversion_agrees_with_oracle(cell):
    rng = np.random.default_rng(11)
    raw = rng.uniform(-1e-2, 1e-2, B.NRAW)
    raw[[8, 9, 12, 13, 14, 17]] = np.abs(raw[[8, 9, 12, 13, 14, 17]])
    p = B.lbm_derive_params(65, 1e6, 0.7, cell)
    q = oracle.derive(65, 1e6, 0.7, cell)
    got = B.lbm_nondimensional(p, raw)
    want = oracle.nondimensional(q, raw)
    for k, v in want.items():
        assert abs(got[k] - v) <= 1e-13 * max(1.0, abs(v)), k


def test_create_rejects_bad_buffers_without_touching_the_gpu():
    lib = B.lib()
    import ctypes
    o = B.lbm_default_opts(U=0.1)
    h = ctypes.c_void_p()
    # misaligned caller buffer
    rc = lib.lbm_create(33, 1e4, 0.71, 0, 1, ctypes.byref(o), ctypes.c_void_p(0x1001), 1 << 30,
                        ctypes.byref(h))
    assert rc == -1
    # buffer too small
    rc = lib.lbm_create(33, 1e4, 0.71, 0, 1, ctypes.byref(o), ctypes.c_void_p(0x100000), 1024,
                        ctypes.byref(h))
    assert rc == -3
    # bad block size
    o.block = 96
    rc = lib.lbm_create(33, 1e4, 0.71, 0, 1, ctypes.byref(o), ctypes.c_void_p(0x100000), 1 << 30,
                        ctypes.byref(h))
    assert rc == -1
    assert lib.lbm_strerror(-5) == b"non-finite result (diverged)"


def test_create_accepts_exactly_the_documented_block_sizes():
    """lbm.h documents opts.block as 64, 128, 192 or 256 (0 = default): those
    create a handle (a fake, never dereferenced device address is enough, as
    lbm_create touches no device memory) and every other value is rejected."""
    import ctypes
    lib = B.lib()
    for block in (0, 64, 128, 192, 256, -64, 1, 32, 96, 255, 320, 512, 1024):
        o = B.lbm_default_opts(U=0.1)
        o.block = block
        h = ctypes.c_void_p()
        rc = lib.lbm_create(33, 1e4, 0.71, 0, 1, ctypes.byref(o), ctypes.c_void_p(0x100000),
                            1 << 30, ctypes.byref(h))
        if block in (0, 64, 128, 192, 256):
            assert rc == 0 and h.value, block
            assert lib.lbm_destroy(h) == 0
        else:
            assert rc == -1 and not h.value, block


def test_warm_start_symbols_exported_and_bound():
    from paper_1903_08882_amd import lws
    text = open(os.path.join(ROOT, "include", "lws.h")).read()
    syms = set(re.findall(r"^LBM_API[^(]*?\b(lws_\w+)\(", text, flags=re.M))
    assert len(syms) >= 15
    lib = lws.lib()
    for s in syms:
        assert hasattr(lib, s), s
        assert hasattr(lws, s) or s == "lws_last_error", s
    assert syms == set(lws._SIG)
    # host-only size queries
    assert lws.lws_packed_elems(8, 16, 0) == 16 * 224
    assert lws.lws_packed_elems(48, 16, 1) == 48 * 448
    assert lws.lws_packed_elems(0, 16, 0) == 0


def test_headers_compile_as_c_and_the_c_example_builds(tmp_path):
    """include/lbm.h and include/lws.h are plain C (C11, -Wall -Wextra
    -Werror); the C example compiles against them and the HIP runtime header."""
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    inc = os.path.join(root, "include")
    src = tmp_path / "h.c"
    src.write_text('#include "lbm.h"\n#include "lws.h"\nint main(void) { return 0; }\n')
    r = subprocess.run(["gcc", "-std=c11", "-Wall", "-Wextra", "-Werror", "-pedantic", "-fsyntax-only",
                        "-I" + inc, str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    demo = os.path.join(root, "paper_1903_08882_amd", "examples", "c_abi_demo.c")
    r = subprocess.run(["gcc", "-std=c11", "-Wall", "-Wextra", "-Werror", "-fsyntax-only",
                        "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + inc, demo],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_product_code_never_reaches_the_oracle():
    """The package (Python and HIP sources) neither imports, loads nor names
    the oracle: only tests, smoke() and the bench's CPU baseline use it."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    pkg = os.path.join(root, "paper_1903_08882_amd")
    offenders = []
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if not f.endswith((".py", ".hip", ".h", ".c")):
                continue
            text = open(os.path.join(dirpath, f)).read()
            if re.search(r"^\s*(import|from)\s+oracle\b|orc_|liborc|oracle\.c", text, re.M):
                offenders.append(f)
    assert not offenders, offenders


def test_hip_build_disables_packed_fp32_instructions():
    """Every HIP compile of the library passes the flag that keeps packed FP32
    instructions out of the generated code."""
    from paper_1903_08882_amd import build as BUILD
    flags = " ".join(BUILD.FLAGS)
    assert "-Xclang -target-feature -Xclang -packed-fp32-ops" in flags
    assert "--offload-arch=gfx950" in flags


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU: --gpus N > 1 (or WORLD_SIZE > 1) exits with
    status 2 and says why, before touching a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2 and "one GPU" in r.stderr
    env = dict(os.environ, WORLD_SIZE="4")
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py")], capture_output=True, text=True,
                       timeout=60, env=env)
    assert r.returncode == 2 and r.stdout == ""
