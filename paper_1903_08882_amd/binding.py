"""Python binding of the C ABI in include/lbm.h (argument marshalling only).

Every function below has the name of the C entry point it calls and does no
arithmetic of the method: the HIP library does all of it.  PyTorch provides
device memory (the state buffer, field and population arrays) and streams
(``torch.cuda.current_stream()`` unless a stream is passed).  The library is
loaded from the package directory; if it is missing, or no GPU is present for
a call that needs one, an error is raised: there is no CPU fallback.
"""
import ctypes
import os

import torch  # loads the HIP runtime the library links against

from .build import LIB_PATH

SIDE_HEATED, RAYLEIGH_BENARD = 0, 1
FP64, FP32, FP16S, FP16C = 0, 1, 2, 3
NRAW, NOBS = 18, 19

CELLS = {"side_heated": SIDE_HEATED, "rayleigh_benard": RAYLEIGH_BENARD}
STORAGES = {"fp64": FP64, "fp32": FP32, "fp16s": FP16S, "fp16c": FP16C}

RAW_NAMES = ["flux_hot", "flux_cold", "flux_hot_mid", "flux_cold_mid", "grad_hot", "grad_cold",
             "grad_hot_mid", "grad_cold_mid", "u2", "w2", "wT", "uT", "eps_u", "eps_T", "drho2",
             "T", "drho", "div2"]
OBS_NAMES = ["Nu_hot", "Nu_cold", "Nu_hot_mid", "Nu_cold_mid", "Nu_hot_fd", "Nu_cold_fd",
             "Nu_hot_mid_fd", "Nu_cold_mid_fd", "Re_rms", "Re_w", "Nu_vol", "eps_u", "eps_T",
             "Nu_kin", "Nu_th", "E", "rms_drho", "mean_T", "rms_div"]

STATUS = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_ERANGE", -3: "LBM_ENOMEM", -4: "LBM_EDEVICE",
          -5: "LBM_EDIVERGED", -6: "LBM_ESTATE", -7: "LBM_EIO"}


class LBMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class lbm_opts(ctypes.Structure):
    _fields_ = [("U", ctypes.c_double), ("T0", ctypes.c_double),
                ("sample_every", ctypes.c_int), ("block", ctypes.c_int),
                ("waves_even", ctypes.c_int), ("waves_odd", ctypes.c_int)]


class lbm_params(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int), ("cell", ctypes.c_int), ("storage", ctypes.c_int),
                ("Ra", ctypes.c_double), ("Pr", ctypes.c_double), ("U", ctypes.c_double),
                ("T0", ctypes.c_double), ("T_hot", ctypes.c_double), ("T_cold", ctypes.c_double),
                ("H", ctypes.c_double), ("dT", ctypes.c_double), ("nu", ctypes.c_double),
                ("kappa", ctypes.c_double), ("gbeta", ctypes.c_double), ("tau_f", ctypes.c_double),
                ("s_e", ctypes.c_double), ("s_q", ctypes.c_double), ("q_k", ctypes.c_double),
                ("q_e", ctypes.c_double), ("q_nu", ctypes.c_double), ("a_T", ctypes.c_double),
                ("wT0", ctypes.c_double), ("wT1", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_SIG = {
    "lbm_default_opts": (None, [ctypes.POINTER(lbm_opts)]),
    "lbm_derive_params": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                         ctypes.c_int, ctypes.POINTER(lbm_opts),
                                         ctypes.POINTER(lbm_params)]),
    "lbm_state_bytes": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]),
    "lbm_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                  ctypes.c_int, ctypes.POINTER(lbm_opts), _P, ctypes.c_size_t,
                                  ctypes.POINTER(_P)]),
    "lbm_destroy": (ctypes.c_int, [_P]),
    "lbm_get_params": (ctypes.c_int, [_P, ctypes.POINTER(lbm_params)]),
    "lbm_set_fields": (ctypes.c_int, [_P, _P, _P]),
    "lbm_get_fields": (ctypes.c_int, [_P, _P, _P]),
    "lbm_set_populations": (ctypes.c_int, [_P, _P, _P]),
    "lbm_get_populations": (ctypes.c_int, [_P, _P, _P]),
    "lbm_step": (ctypes.c_int, [_P, ctypes.c_int64, _P]),
    "lbm_time": (ctypes.c_int64, [_P]),
    "lbm_observables_raw": (ctypes.c_int, [_P, _P, _D]),
    "lbm_nusselt_profile": (ctypes.c_int, [_P, _P, _D]),
    "lbm_device_copy": (ctypes.c_int, [_P, _P, ctypes.c_size_t, _P]),
    "lbm_observables": (ctypes.c_int, [_P, _P, _D, _D, _D, _D]),
    "lbm_nondimensional": (ctypes.c_int, [ctypes.POINTER(lbm_params), _D, _D]),
    "lbm_averages": (ctypes.c_int, [_P, _P, _D, ctypes.POINTER(ctypes.c_int64)]),
    "lbm_reset_averages": (ctypes.c_int, [_P, _P]),
    "lbm_residual": (ctypes.c_int, [_P, _P, _D, _D, _D]),
    "lbm_run_to_steady": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_double, ctypes.c_int64, _P,
                                         ctypes.POINTER(ctypes.c_int64), _D, _D, ctypes.c_int64]),
    "lbm_save": (ctypes.c_int, [_P, ctypes.c_char_p, _P]),
    "lbm_load": (ctypes.c_int, [_P, ctypes.c_char_p, _P]),
    "lbm_centerline_peaks": (ctypes.c_int, [_P, _P, _D]),
    "lbm_resample_fields": (ctypes.c_int, [_P, ctypes.c_int, _P, _P]),
    "lbm_autotune": (ctypes.c_int, [_P, _P, ctypes.c_int, ctypes.POINTER(ctypes.c_int), _D]),
    "lbm_batch_state_bytes": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                                             ctypes.POINTER(ctypes.c_size_t)]),
    "lbm_batch_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int), _D, _D,
                                        ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                                        ctypes.POINTER(lbm_opts), _P, ctypes.c_size_t,
                                        ctypes.POINTER(_P)]),
    "lbm_batch_destroy": (ctypes.c_int, [_P]),
    "lbm_batch_cavity": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(_P)]),
    "lbm_batch_step": (ctypes.c_int, [_P, ctypes.c_int64, _P]),
    "lbm_batch_run_to_steady": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_double, ctypes.c_int64, _P,
                                               ctypes.POINTER(ctypes.c_int64), _D]),
    "lbm_batch_autotune": (ctypes.c_int, [_P, _P, ctypes.c_int, ctypes.POINTER(ctypes.c_int), _D]),
    "lbm_batch_last_error": (ctypes.c_char_p, [_P]),
    "lbm_profile": (ctypes.c_int, [_P, ctypes.c_int]),
    "lbm_profile_read": (ctypes.c_int, [_P, _D, ctypes.POINTER(ctypes.c_int64)]),
    "lbm_last_error": (ctypes.c_char_p, [_P]),
    "lbm_strerror": (ctypes.c_char_p, [ctypes.c_int]),
}


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1903_08882_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIG.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc, h=None):
    if rc != 0:
        msg = lib().lbm_last_error(h).decode() if h else lib().lbm_strerror(rc).decode()
        raise LBMError(rc, msg or lib().lbm_strerror(rc).decode())


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_ptr(t, dtype=torch.float64, numel=None):
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"expected a contiguous {dtype} CUDA tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"expected {numel} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _d(arr):
    return arr.ctypes.data_as(_D) if hasattr(arr, "ctypes") else arr


# --------------------------------------------------------------------------
# Entry points (same names as the C ABI)
# --------------------------------------------------------------------------

def lbm_default_opts(**kw):
    o = lbm_opts()
    lib().lbm_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if v is not None:
            setattr(o, k, v)
    return o


def lbm_derive_params(N, Ra, Pr, cell="side_heated", storage="fp32", opts=None):
    p = lbm_params()
    o = opts if opts is not None else lbm_default_opts()
    _check(lib().lbm_derive_params(int(N), float(Ra), float(Pr), CELLS.get(cell, cell),
                                   STORAGES.get(storage, storage), ctypes.byref(o), ctypes.byref(p)))
    return p


def lbm_state_bytes(N, storage="fp32"):
    b = ctypes.c_size_t()
    _check(lib().lbm_state_bytes(int(N), STORAGES.get(storage, storage), ctypes.byref(b)))
    return b.value


class Handle:
    """An lbm_t* with the torch buffer that backs it (kept alive with it)."""

    def __init__(self, ptr, buf, N):
        self.ptr = ptr
        self.buf = buf
        self.N = N
        self.V = N ** 3

    def __del__(self):
        if getattr(self, "ptr", None) and _lib is not None and not getattr(self, "owned_by_batch", False):
            _lib.lbm_destroy(self.ptr)
            self.ptr = None


def lbm_create(N, Ra, Pr, cell="side_heated", storage="fp32", opts=None, device=None):
    """Allocate the state buffer with torch and create a handle."""
    nbytes = lbm_state_bytes(N, storage)
    buf = torch.empty(nbytes, dtype=torch.uint8, device=device or "cuda")
    o = opts if opts is not None else lbm_default_opts()
    h = ctypes.c_void_p()
    _check(lib().lbm_create(int(N), float(Ra), float(Pr), CELLS.get(cell, cell),
                            STORAGES.get(storage, storage), ctypes.byref(o),
                            ctypes.c_void_p(buf.data_ptr()), nbytes, ctypes.byref(h)))
    return Handle(h, buf, int(N))


def lbm_destroy(h):
    if h.ptr:
        _check(lib().lbm_destroy(h.ptr))
        h.ptr = None


def lbm_get_params(h):
    p = lbm_params()
    _check(lib().lbm_get_params(h.ptr, ctypes.byref(p)), h.ptr)
    return p


def lbm_set_fields(h, uvwT, stream=None):
    """uvwT: CUDA float64 tensor of 4*N^3 elements (u, v, w, T planes, x fastest)."""
    _check(lib().lbm_set_fields(h.ptr, _dev_ptr(uvwT, numel=4 * h.V), _stream(stream)), h.ptr)


def lbm_get_fields(h, out=None, stream=None):
    out = out if out is not None else torch.empty(5 * h.V, dtype=torch.float64, device=h.buf.device)
    _check(lib().lbm_get_fields(h.ptr, _dev_ptr(out, numel=5 * h.V), _stream(stream)), h.ptr)
    return out


def lbm_set_populations(h, pop, stream=None):
    _check(lib().lbm_set_populations(h.ptr, _dev_ptr(pop, numel=26 * h.V), _stream(stream)), h.ptr)


def lbm_get_populations(h, out=None, stream=None):
    out = out if out is not None else torch.empty(26 * h.V, dtype=torch.float64, device=h.buf.device)
    _check(lib().lbm_get_populations(h.ptr, _dev_ptr(out, numel=26 * h.V), _stream(stream)), h.ptr)
    return out


def lbm_step(h, n=1, stream=None):
    _check(lib().lbm_step(h.ptr, int(n), _stream(stream)), h.ptr)


def lbm_time(h):
    return int(lib().lbm_time(h.ptr))


def lbm_observables_raw(h, stream=None):
    raw = (ctypes.c_double * NRAW)()
    _check(lib().lbm_observables_raw(h.ptr, _stream(stream), raw), h.ptr)
    return list(raw)


def lbm_device_copy(dst, src, stream=None):
    """Reference streaming copy of the CUDA tensor src into dst (same byte
    size, a multiple of 16), asynchronous on stream."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes or not (src.is_cuda and dst.is_cuda):
        raise LBMError(-1, "lbm_device_copy needs two CUDA tensors of the same byte size")
    _check(lib().lbm_device_copy(dst.data_ptr(), src.data_ptr(), nbytes, _stream(stream)))


def lbm_nusselt_profile(h, stream=None):
    """Plane-averaged Nu on the N node planes across the cell (list of N)."""
    n = lbm_get_params(h).N
    out = (ctypes.c_double * n)()
    _check(lib().lbm_nusselt_profile(h.ptr, _stream(stream), out), h.ptr)
    return list(out)


def lbm_observables(h, stream=None):
    """(Nu, Re, eps_u, eps_T) of the current state, nondimensional."""
    v = [ctypes.c_double() for _ in range(4)]
    _check(lib().lbm_observables(h.ptr, _stream(stream), *[ctypes.byref(x) for x in v]), h.ptr)
    return tuple(x.value for x in v)


def lbm_nondimensional(params, raw):
    r = (ctypes.c_double * NRAW)(*raw)
    out = (ctypes.c_double * NOBS)()
    _check(lib().lbm_nondimensional(ctypes.byref(params), r, out))
    return dict(zip(OBS_NAMES, list(out)))


def lbm_averages(h, stream=None):
    raw = (ctypes.c_double * NRAW)()
    cnt = ctypes.c_int64()
    _check(lib().lbm_averages(h.ptr, _stream(stream), raw, ctypes.byref(cnt)), h.ptr)
    return list(raw), cnt.value


def lbm_reset_averages(h, stream=None):
    _check(lib().lbm_reset_averages(h.ptr, _stream(stream)), h.ptr)


def lbm_residual(h, stream=None):
    """(max |dT|, rel L1 of T, rel L2 of u) against the previous call."""
    v = [ctypes.c_double() for _ in range(3)]
    _check(lib().lbm_residual(h.ptr, _stream(stream), *[ctypes.byref(x) for x in v]), h.ptr)
    return tuple(x.value for x in v)


def lbm_run_to_steady(h, check_every=1000, tol_max_dT=1e-8, max_steps=10**6, stream=None,
                      history_len=0):
    """(steps taken, final max |dT|, residual history) of the steady-state loop."""
    steps = ctypes.c_int64()
    r = ctypes.c_double()
    hist = (ctypes.c_double * max(history_len, 1))()
    _check(lib().lbm_run_to_steady(h.ptr, int(check_every), float(tol_max_dT), int(max_steps),
                                   _stream(stream), ctypes.byref(steps), ctypes.byref(r),
                                   hist if history_len else None, int(history_len)), h.ptr)
    nchk = -(-steps.value // int(check_every))
    return steps.value, r.value, list(hist)[:min(history_len, nchk)]


def lbm_save(h, path, stream=None):
    """Write the handle's state to the checkpoint file `path`."""
    _check(lib().lbm_save(h.ptr, os.fsencode(path), _stream(stream)), h.ptr)


def lbm_load(h, path, stream=None):
    """Restore a checkpoint written by lbm_save into a handle with the same set-up."""
    _check(lib().lbm_load(h.ptr, os.fsencode(path), _stream(stream)), h.ptr)


def lbm_centerline_peaks(h, stream=None):
    """dict: u_max, z of u_max, w_max, x of w_max (nondimensional), E."""
    out = (ctypes.c_double * 5)()
    _check(lib().lbm_centerline_peaks(h.ptr, _stream(stream), out), h.ptr)
    return dict(zip(["u_max", "u_max_z", "w_max", "w_max_x", "E"], list(out)))


def lbm_resample_fields(h, M, out=None, stream=None):
    """(u, v, w, T) on M^3 node-centred points: CUDA float32 tensor [4][M^3]."""
    out = out if out is not None else torch.empty(4 * M ** 3, dtype=torch.float32, device=h.buf.device)
    _check(lib().lbm_resample_fields(h.ptr, int(M), _dev_ptr(out, torch.float32, 4 * M ** 3),
                                     _stream(stream)), h.ptr)
    return out


def lbm_autotune(h, steps_per_candidate=20, stream=None):
    """(best block size, its mean step time in ms; 0 when taken from the cache)."""
    blk = ctypes.c_int()
    ms = ctypes.c_double()
    _check(lib().lbm_autotune(h.ptr, _stream(stream), int(steps_per_candidate), ctypes.byref(blk),
                              ctypes.byref(ms)), h.ptr)
    return blk.value, ms.value


class Batch:
    """An lbm_batch_t* with its torch buffer and per-cavity handles."""

    def __init__(self, ptr, buf, Ns):
        self.ptr = ptr
        self.buf = buf
        self.Ns = list(Ns)
        self.cavities = []
        for k, N in enumerate(self.Ns):
            hp = ctypes.c_void_p()
            _bcheck(lib().lbm_batch_cavity(ptr, k, ctypes.byref(hp)), ptr)
            c = Handle(hp, buf, N)
            c.owned_by_batch = True
            self.cavities.append(c)

    def __del__(self):
        if getattr(self, "ptr", None) and _lib is not None:
            for c in self.cavities:
                c.ptr = None           # destroyed with the batch
            _lib.lbm_batch_destroy(self.ptr)
            self.ptr = None


def _bcheck(rc, b=None):
    if rc != 0:
        msg = lib().lbm_batch_last_error(b).decode() if b else lib().lbm_strerror(rc).decode()
        raise LBMError(rc, msg or lib().lbm_strerror(rc).decode())


def _ints(v):
    return (ctypes.c_int * len(v))(*[int(x) for x in v])


def _dbls(v):
    return (ctypes.c_double * len(v))(*[float(x) for x in v])


def lbm_batch_state_bytes(Ns, storage="fp32"):
    b = ctypes.c_size_t()
    _check(lib().lbm_batch_state_bytes(len(Ns), _ints(Ns), STORAGES.get(storage, storage),
                                       ctypes.byref(b)))
    return b.value


def lbm_batch_create(Ns, Ras, Prs, cells, storage="fp32", opts=None, device=None):
    nbytes = lbm_batch_state_bytes(Ns, storage)
    buf = torch.empty(nbytes, dtype=torch.uint8, device=device or "cuda")
    o = opts if opts is not None else lbm_default_opts()
    b = ctypes.c_void_p()
    cells = [CELLS.get(c, c) for c in cells]
    _check(lib().lbm_batch_create(len(Ns), _ints(Ns), _dbls(Ras), _dbls(Prs), _ints(cells),
                                  STORAGES.get(storage, storage), ctypes.byref(o),
                                  ctypes.c_void_p(buf.data_ptr()), nbytes, ctypes.byref(b)))
    return Batch(b, buf, Ns)


def lbm_batch_cavity(b, k):
    """The handle of cavity k (owned by the batch)."""
    return b.cavities[k]


def lbm_batch_destroy(b):
    if b.ptr:
        for c in b.cavities:
            c.ptr = None
        _bcheck(lib().lbm_batch_destroy(b.ptr))
        b.ptr = None


def lbm_batch_step(b, n=1, stream=None):
    _bcheck(lib().lbm_batch_step(b.ptr, int(n), _stream(stream)), b.ptr)


def lbm_batch_run_to_steady(b, check_every=1000, tol_max_dT=1e-8, max_steps=10**6, stream=None):
    """(steps each cavity took, last max |dT| of each cavity)."""
    K = len(b.Ns)
    steps = (ctypes.c_int64 * K)()
    res = (ctypes.c_double * K)()
    _bcheck(lib().lbm_batch_run_to_steady(b.ptr, int(check_every), float(tol_max_dT), int(max_steps),
                                          _stream(stream), steps, res), b.ptr)
    return list(steps), list(res)


def lbm_batch_autotune(b, steps_per_candidate=20, stream=None):
    blk = ctypes.c_int()
    ms = ctypes.c_double()
    _bcheck(lib().lbm_batch_autotune(b.ptr, _stream(stream), int(steps_per_candidate),
                                     ctypes.byref(blk), ctypes.byref(ms)), b.ptr)
    return blk.value, ms.value


def lbm_profile(h, enable=True):
    _check(lib().lbm_profile(h.ptr, int(bool(enable))), h.ptr)


def lbm_profile_read(h):
    ms = ctypes.c_double()
    k = ctypes.c_int64()
    _check(lib().lbm_profile_read(h.ptr, ctypes.byref(ms), ctypes.byref(k)), h.ptr)
    return ms.value, k.value
