"""Plain FP64 CPU oracle of the coupled D3Q19-MRT / D3Q7-MRT thermal lattice
Boltzmann method (Xu, Shi & Xi 2019, arXiv:1903.08882).

TEST INFRASTRUCTURE ONLY: the correctness reference the HIP library is
compared against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import it; the product path never does.  It
shares no code with the GPU library (``oracle.c`` holds every constant and
formula on its own); this module is argument marshalling around it.

Array layout: population q (0..18 = f_0..f_18, 19..25 = g_0..g_6) of node
(x, y, z) is ``pop[q, z, y, x]``; macro planes are ``[rho, u, v, w, T]``.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIBPATH = os.path.join(_HERE, "liboracle.so")
_lib = None

SIDE_HEATED = 0
RAYLEIGH_BENARD = 1
NRAW = 18


def build():
    """Compile oracle.c into liboracle.so (plain gcc, FP64, OpenMP)."""
    tmp = _LIBPATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                           _SRC, "-o", tmp, "-lm"])
    os.replace(tmp, _LIBPATH)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIBPATH):
            build()
        L = ctypes.CDLL(_LIBPATH)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(Params)
        L.orc_derive.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                 ctypes.c_double, ctypes.c_double, pp]
        L.orc_derive.restype = ctypes.c_int
        L.orc_step.argtypes = [pp, dp, dp, dp]
        L.orc_init_fields.argtypes = [pp, dp, dp, dp]
        L.orc_macro_fields.argtypes = [pp, dp, dp]
        L.orc_observables.argtypes = [pp, dp, dp, dp]
        L.orc_residual.argtypes = [pp, dp, dp, dp]
        L.orc_nusselt_profile.argtypes = [pp, dp, dp]
        L.orc_collide.argtypes = [pp, dp, dp, dp, dp, dp]
        L.orc_macros.argtypes = [pp, dp, dp, dp, dp]
        L.orc_feq.argtypes = [ctypes.c_double, dp, dp]
        L.orc_geq.argtypes = [pp, ctypes.c_double, dp, dp]
        L.orc_meq.argtypes = [ctypes.c_double, dp, dp]
        L.orc_neq.argtypes = [pp, ctypes.c_double, dp, dp]
        L.orc_force_moments.argtypes = [dp, dp, dp]
        L.orc_relaxation.argtypes = [pp, dp, dp]
        L.orc_matrix_M.argtypes = [dp]
        L.orc_matrix_N.argtypes = [dp]
        L.orc_invert.argtypes = [ctypes.c_int, dp, dp]
        L.orc_invert.restype = ctypes.c_int
        L.orc_velocities19.argtypes = [ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), dp]
        L.orc_velocities7.argtypes = [ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
        L.orc_fd_derivative.argtypes = [ctypes.c_int, dp, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                        ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int]
        L.orc_fd_derivative.restype = ctypes.c_double
        L.orc_threads.restype = ctypes.c_int
        _lib = L
    return _lib


class Params(ctypes.Structure):
    """Mirror of ``orc_params`` in oracle.c."""
    _fields_ = [("N", ctypes.c_int), ("cell", ctypes.c_int),
                ("Ra", ctypes.c_double), ("Pr", ctypes.c_double), ("U", ctypes.c_double),
                ("T0", ctypes.c_double), ("T_hot", ctypes.c_double), ("T_cold", ctypes.c_double),
                ("H", ctypes.c_double), ("dT", ctypes.c_double),
                ("nu", ctypes.c_double), ("kappa", ctypes.c_double), ("gbeta", ctypes.c_double),
                ("tau_f", ctypes.c_double), ("s_e", ctypes.c_double), ("s_q", ctypes.c_double),
                ("q_k", ctypes.c_double), ("q_e", ctypes.c_double), ("q_nu", ctypes.c_double),
                ("a_T", ctypes.c_double), ("wT0", ctypes.c_double), ("wT1", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def derive(N, Ra, Pr, cell=SIDE_HEATED, U=0.1 / np.sqrt(3.0), T0=0.0):
    """Lattice parameters for (N, Ra, Pr, U); raises ValueError when invalid."""
    p = Params()
    rc = lib().orc_derive(int(N), float(Ra), float(Pr), int(cell), float(U), float(T0),
                          ctypes.byref(p))
    if rc != 0:
        raise ValueError(f"orc_derive failed ({rc}) for N={N} Ra={Ra} Pr={Pr} U={U}")
    return p


def threads():
    """OpenMP threads the oracle's whole-lattice loops run on."""
    return int(lib().orc_threads())


def matrix_M():
    M = np.zeros(19 * 19)
    lib().orc_matrix_M(_dp(M))
    return M.reshape(19, 19)


def matrix_N():
    Nm = np.zeros(7 * 7)
    lib().orc_matrix_N(_dp(Nm))
    return Nm.reshape(7, 7)


def invert(A):
    A = _f64(A)
    out = np.zeros_like(A)
    if not lib().orc_invert(A.shape[0], _dp(A), _dp(out)):
        raise np.linalg.LinAlgError("singular")
    return out


def velocities19():
    e = np.zeros(57, dtype=np.int32)
    opp = np.zeros(19, dtype=np.int32)
    w = np.zeros(19)
    lib().orc_velocities19(e.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                           opp.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(w))
    return e.reshape(19, 3), opp, w


def velocities7():
    e = np.zeros(21, dtype=np.int32)
    opp = np.zeros(7, dtype=np.int32)
    lib().orc_velocities7(e.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                          opp.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return e.reshape(7, 3), opp


def feq(rho, u):
    out = np.zeros(19)
    lib().orc_feq(float(rho), _dp(_f64(u)), _dp(out))
    return out


def geq(p, T, u):
    out = np.zeros(7)
    lib().orc_geq(ctypes.byref(p), float(T), _dp(_f64(u)), _dp(out))
    return out


def meq(rho, u):
    out = np.zeros(19)
    lib().orc_meq(float(rho), _dp(_f64(u)), _dp(out))
    return out


def neq(p, T, u):
    out = np.zeros(7)
    lib().orc_neq(ctypes.byref(p), float(T), _dp(_f64(u)), _dp(out))
    return out


def force_moments(u, F):
    out = np.zeros(19)
    lib().orc_force_moments(_dp(_f64(u)), _dp(_f64(F)), _dp(out))
    return out


def relaxation(p):
    S = np.zeros(19)
    Qd = np.zeros(7)
    lib().orc_relaxation(ctypes.byref(p), _dp(S), _dp(Qd))
    return S, Qd


def macros(p, f, g):
    mc = np.zeros(5)
    F = np.zeros(3)
    lib().orc_macros(ctypes.byref(p), _dp(_f64(f)), _dp(_f64(g)), _dp(mc), _dp(F))
    return mc, F


def collide(p, f, g):
    """Post-collision (f+, g+) and the node's macros {rho, u, v, w, T}."""
    fp = np.zeros(19)
    gp = np.zeros(7)
    mc = np.zeros(5)
    lib().orc_collide(ctypes.byref(p), _dp(_f64(f)), _dp(_f64(g)), _dp(fp), _dp(gp), _dp(mc))
    return fp, gp, mc


def fd_derivative(phi, axis, c, wall_lo=0.0, wall_hi=0.0, adiab_lo=False, adiab_hi=False):
    phi = _f64(phi)
    N = phi.shape[0]
    cc = (ctypes.c_int * 3)(*[int(v) for v in c])
    return lib().orc_fd_derivative(N, _dp(phi), int(axis), cc, float(wall_lo), float(wall_hi),
                                   int(adiab_lo), int(adiab_hi))


class Oracle:
    """A whole lattice advanced by the oracle (two population arrays)."""

    def __init__(self, N, Ra, Pr, cell=SIDE_HEATED, U=0.1 / np.sqrt(3.0), T0=0.0, params=None):
        self.p = params if params is not None else derive(N, Ra, Pr, cell, U, T0)
        self.N = self.p.N
        self.V = self.N ** 3
        self.pop = np.zeros((26, self.V))
        self._tmp = np.zeros((26, self.V))
        self.flux = np.zeros(4)
        self.t = 0

    def init_fields(self, uvwT, rho=None):
        """f = f^eq(rho, u), g = g^eq(T, u); uvwT has shape (4, N, N, N) [z][y][x]."""
        f = _f64(np.reshape(uvwT, (4, self.V)))
        r = None if rho is None else _f64(np.reshape(rho, self.V))
        lib().orc_init_fields(ctypes.byref(self.p), _dp(f), None if r is None else _dp(r),
                              _dp(self.pop))
        self.flux[:] = 0.0
        self.t = 0

    def set_populations(self, pop):
        self.pop[:] = np.reshape(pop, (26, self.V))
        self.flux[:] = 0.0

    def populations(self):
        return self.pop.reshape(26, self.N, self.N, self.N).copy()

    def step(self, n=1):
        for _ in range(int(n)):
            lib().orc_step(ctypes.byref(self.p), _dp(self.pop), _dp(self._tmp), _dp(self.flux))
            self.pop, self._tmp = self._tmp, self.pop
            self.t += 1

    def macro(self):
        out = np.zeros((5, self.V))
        lib().orc_macro_fields(ctypes.byref(self.p), _dp(self.pop), _dp(out))
        return out

    def observables_raw(self, macro=None):
        m = self.macro() if macro is None else _f64(macro)
        r = np.zeros(NRAW)
        lib().orc_observables(ctypes.byref(self.p), _dp(m), _dp(self.flux), _dp(r))
        return r

    def nusselt_profile(self, macro=None):
        """Plane-averaged Nu on the N node planes across the cell (x for the
        side-heated cell, z for Rayleigh-Benard), oracle.c orc_nusselt_profile."""
        m = self.macro() if macro is None else _f64(macro)
        out = np.zeros(self.N)
        lib().orc_nusselt_profile(ctypes.byref(self.p), _dp(m), _dp(out))
        return out

    def residual(self, macro_old, macro=None):
        m = self.macro() if macro is None else _f64(macro)
        res = np.zeros(3)
        lib().orc_residual(ctypes.byref(self.p), _dp(m), _dp(_f64(macro_old)), _dp(res))
        return res


def nondimensional(p, r):
    """Nusselt, Reynolds and dissipation numbers from a raw vector (Sec. 3, 4).

    H = N, dT = 1, U the free-fall velocity; u* = u/U, T* = T/dT, lengths in H.
    """
    H, U, dT, nu, kappa = p.H, p.U, p.dT, p.nu, p.kappa
    s = np.sqrt(p.Ra * p.Pr)
    eps_u = r[12] * H / U ** 3
    eps_T = r[13] * H / (U * dT ** 2)
    vt = r[10] if p.cell == RAYLEIGH_BENARD else r[11]
    return {
        "Nu_hot": r[0] * H / (kappa * dT), "Nu_cold": -r[1] * H / (kappa * dT),
        "Nu_hot_mid": r[2] * H / (kappa * dT), "Nu_cold_mid": -r[3] * H / (kappa * dT),
        "Nu_hot_fd": r[4] * H / dT, "Nu_cold_fd": -r[5] * H / dT,
        "Nu_hot_mid_fd": r[6] * H / dT, "Nu_cold_mid_fd": -r[7] * H / dT,
        "Re_rms": np.sqrt(r[8]) * H / nu, "Re_w": np.sqrt(r[9]) * H / nu,
        "Nu_vol": 1.0 + s * vt / (U * dT),
        "eps_u": eps_u, "eps_T": eps_T,
        "Nu_kin": 1.0 + s * eps_u, "Nu_th": s * eps_T,
        "E": 0.5 * r[8] / U ** 2,
        "rms_drho": np.sqrt(r[14]), "mean_T": r[15],
        "rms_div": np.sqrt(r[17]) * H / U,
    }
