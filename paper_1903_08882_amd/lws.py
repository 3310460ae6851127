"""ctypes binding of the warm-start network ABI (include/lws.h): the same
names and arguments, marshalled; every computation runs in the library.

Device arrays are torch tensors: bfloat16 operands are carried as int16
tensors holding the raw bits, FP32/FP64 arrays as float32/float64 tensors.
"""
import ctypes

import numpy as np
import torch

from .binding import LBMError, lib as _lbm_lib, _stream

_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)


class lws_grid(ctypes.Structure):
    _fields_ = [("B", ctypes.c_int), ("D", ctypes.c_int), ("H", ctypes.c_int), ("W", ctypes.c_int)]


_SIG = {
    "lws_packed_elems": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "lws_pack_weights": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P, _P]),
    "lws_conv3d_forward": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, _P, ctypes.c_int, _P, lws_grid, _P]),
    "lws_conv3d_backward_data": (ctypes.c_int, [_P, ctypes.c_int, _P, ctypes.c_int, _P, lws_grid, _P]),
    "lws_wgrad_work_bytes": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_int, lws_grid]),
    "lws_conv3d_backward_weight": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, _P, ctypes.c_int, _P,
                                                  lws_grid, _P, ctypes.c_size_t, _P]),
    "lws_conv3d_backward_weight_noalloc": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, _P, ctypes.c_int,
                                                          _P, lws_grid, _P]),
    "lws_upsample_fields": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                           _P, _P]),
    "lws_net_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                      ctypes.POINTER(_P)]),
    "lws_net_destroy": (ctypes.c_int, [_P]),
    "lws_net_param_count": (ctypes.c_int64, [_P]),
    "lws_net_set_params": (ctypes.c_int, [_P, _P]),
    "lws_net_get_params": (ctypes.c_int, [_P, _P]),
    "lws_net_forward": (ctypes.c_int, [_P, ctypes.c_int, _D, _P, _P]),
    "lws_net_loss_grad": (ctypes.c_int, [_P, ctypes.c_int, _D, _P, _D, _D, _P]),
    "lws_net_get_grad": (ctypes.c_int, [_P, _P]),
    "lws_net_adam": (ctypes.c_int, [_P, ctypes.c_double, _P]),
    "lws_last_error": (ctypes.c_char_p, [_P]),
}
_ready = False


def lib():
    global _ready
    L = _lbm_lib()
    if not _ready:
        for name, (res, args) in _SIG.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _ready = True
    return L


def _check(rc, net=None):
    if rc != 0:
        msg = lib().lws_last_error(net).decode() if net else lib().lbm_strerror(rc).decode()
        raise LBMError(rc, msg or lib().lbm_strerror(rc).decode())


def _ptr(t, dtype, numel):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"expected a contiguous {dtype} CUDA tensor")
    if t.numel() < numel:
        raise ValueError(f"tensor has {t.numel()} elements, {numel} needed")
    return ctypes.c_void_p(t.data_ptr())


def _grid(g):
    return lws_grid(*[int(v) for v in g])


def _vox(g):
    return int(g[0]) * int(g[1]) * int(g[2]) * int(g[3])


def lws_packed_elems(cin, cout, for_data_grad=0):
    return int(lib().lws_packed_elems(int(cin), int(cout), int(for_data_grad)))


def lws_pack_weights(w, cin, cout, for_data_grad=0, out=None, stream=None):
    n = lws_packed_elems(cin, cout, for_data_grad)
    out = out if out is not None else torch.empty(n, dtype=torch.int16, device=w.device)
    _check(lib().lws_pack_weights(_ptr(w, torch.float32, 27 * cin * cout), int(cin), int(cout),
                                  int(for_data_grad), _ptr(out, torch.int16, n), _stream(stream)))
    return out


def lws_conv3d_forward(x, x_shared, cin, packed, cout, grid, out=None, stream=None):
    """grid = (B, D, H, W); x is int16 (bfloat16 bits) channels-last."""
    V = _vox(grid)
    out = out if out is not None else torch.empty(V * cout, dtype=torch.float32, device=x.device)
    nx = (V // int(grid[0]) if x_shared else V) * cin
    _check(lib().lws_conv3d_forward(_ptr(x, torch.int16, nx), int(bool(x_shared)), int(cin),
                                    _ptr(packed, torch.int16, lws_packed_elems(cin, cout, 0)), int(cout),
                                    _ptr(out, torch.float32, V * cout), _grid(grid), _stream(stream)))
    return out


def lws_conv3d_backward_data(dz, cout, packed, cin, grid, out=None, stream=None):
    V = _vox(grid)
    out = out if out is not None else torch.empty(V * cin, dtype=torch.float32, device=dz.device)
    _check(lib().lws_conv3d_backward_data(_ptr(dz, torch.int16, V * cout), int(cout),
                                          _ptr(packed, torch.int16, lws_packed_elems(cin, cout, 1)), int(cin),
                                          _ptr(out, torch.float32, V * cin), _grid(grid), _stream(stream)))
    return out


def lws_wgrad_work_bytes(cin, cout, grid):
    return int(lib().lws_wgrad_work_bytes(int(cin), int(cout), _grid(grid)))


def lws_conv3d_backward_weight(x, x_shared, cin, dz, cout, grid, out=None, work=None, stream=None):
    V = _vox(grid)
    out = out if out is not None else torch.empty(27 * cin * cout, dtype=torch.float32, device=dz.device)
    wb = lws_wgrad_work_bytes(cin, cout, grid)
    work = work if work is not None else torch.empty(max(wb, 4), dtype=torch.uint8, device=dz.device)
    nx = (V // int(grid[0]) if x_shared else V) * cin
    _check(lib().lws_conv3d_backward_weight(_ptr(x, torch.int16, nx), int(bool(x_shared)), int(cin),
                                            _ptr(dz, torch.int16, V * cout), int(cout),
                                            _ptr(out, torch.float32, 27 * cin * cout), _grid(grid),
                                            _ptr(work, torch.uint8, wb), ctypes.c_size_t(work.numel()),
                                            _stream(stream)))
    return out


def lws_conv3d_backward_weight_noalloc(x, x_shared, cin, dz, cout, grid, out, stream=None):
    """As lws_conv3d_backward_weight with the library's own scratch array
    instead of a workspace; out must be given (nothing is allocated)."""
    V = _vox(grid)
    nx = (V // int(grid[0]) if x_shared else V) * cin
    _check(lib().lws_conv3d_backward_weight_noalloc(_ptr(x, torch.int16, nx), int(bool(x_shared)), int(cin),
                                                    _ptr(dz, torch.int16, V * cout), int(cout),
                                                    _ptr(out, torch.float32, 27 * cin * cout), _grid(grid),
                                                    _stream(stream)))
    return out


def lws_upsample_fields(pred, M, ld, N, cell, U, T_hot, T_cold, out=None, stream=None, symmetrize=False):
    cellv = {"side_heated": 0, "rayleigh_benard": 1}.get(cell, cell)
    out = out if out is not None else torch.empty(4 * N ** 3, dtype=torch.float64, device=pred.device)
    _check(lib().lws_upsample_fields(_ptr(pred, torch.float32, M ** 3 * ld), int(M), int(ld), int(N), int(cellv),
                                     float(U), float(T_hot), float(T_cold), int(bool(symmetrize)),
                                     _ptr(out, torch.float64, 4 * N ** 3),
                                     _stream(stream)))
    return out


class Net:
    def __init__(self, ptr, M, max_batch, ch):
        self.ptr, self.M, self.max_batch, self.ch = ptr, M, max_batch, tuple(ch)

    def __del__(self):
        if getattr(self, "ptr", None):
            try:
                lib().lws_net_destroy(self.ptr)
            except Exception:       # interpreter shutdown
                pass
            self.ptr = None


def lws_net_create(M, max_batch=8, ch=(16, 32, 64)):
    c = (ctypes.c_int * 3)(*ch)
    p = _P()
    _check(lib().lws_net_create(int(M), int(max_batch), c, ctypes.byref(p)))
    return Net(p, M, max_batch, ch)


def lws_net_destroy(net):
    if net.ptr:
        _check(lib().lws_net_destroy(net.ptr))
        net.ptr = None


def lws_net_param_count(net):
    return int(lib().lws_net_param_count(net.ptr))


def lws_net_set_params(net, host):
    a = np.ascontiguousarray(host, dtype=np.float32)
    if a.size != lws_net_param_count(net):
        raise ValueError("parameter vector of the wrong length")
    _check(lib().lws_net_set_params(net.ptr, a.ctypes.data_as(_P)), net.ptr)


def lws_net_get_params(net):
    a = np.empty(lws_net_param_count(net), dtype=np.float32)
    _check(lib().lws_net_get_params(net.ptr, a.ctypes.data_as(_P)), net.ptr)
    return a


def lws_net_get_grad(net):
    a = np.empty(lws_net_param_count(net), dtype=np.float32)
    _check(lib().lws_net_get_grad(net.ptr, a.ctypes.data_as(_P)), net.ptr)
    return a


def _ra_pr(ra_pr):
    a = np.ascontiguousarray(np.asarray(ra_pr, dtype=np.float64).reshape(-1, 2))
    return a, a.ctypes.data_as(_D)


def lws_net_forward(net, ra_pr, out=None, stream=None):
    a, p = _ra_pr(ra_pr)
    B = a.shape[0]
    n = B * net.M ** 3 * 8
    out = out if out is not None else torch.empty(n, dtype=torch.float32, device="cuda")
    _check(lib().lws_net_forward(net.ptr, B, p, _ptr(out, torch.float32, n), _stream(stream)), net.ptr)
    return out


def lws_net_loss_grad(net, ra_pr, target, scale=None, stream=None):
    a, p = _ra_pr(ra_pr)
    B = a.shape[0]
    sc = None
    if scale is not None:
        sc = np.ascontiguousarray(np.asarray(scale, dtype=np.float64).reshape(B, 4))
    loss = ctypes.c_double()
    _check(lib().lws_net_loss_grad(net.ptr, B, p, _ptr(target, torch.float32, B * 4 * net.M ** 3),
                                   sc.ctypes.data_as(_D) if sc is not None else None, ctypes.byref(loss),
                                   _stream(stream)), net.ptr)
    return loss.value


def lws_net_adam(net, lr, stream=None):
    _check(lib().lws_net_adam(net.ptr, float(lr), _stream(stream)), net.ptr)
