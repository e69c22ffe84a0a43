"""TEST INFRASTRUCTURE ONLY: ctypes wrapper around the FP64 CPU oracle.

The oracle (``dmrt_oracle.c``) is a plain, slow, double-precision CPU
implementation of the double-MRT thermal lattice Boltzmann step of Li, Yang &
Zhang (arXiv:1601.04633), Sections 3.1-3.2, Eqs. 22-45.  Only the tests, the
smoke check and the CPU-baseline leg of the benchmark may use it.  It never
imports the GPU package and the GPU package never imports it.

State convention: the oracle stores the *pre-collision* populations f(t), g(t)
as arrays of structures, ``f[(y*n + x)*9 + i]`` and ``g[(y*n + x)*5 + i]``,
with f stored as the deviation whose sum is the density deviation (Eq. 33).

Parity status of every function here: pinned by ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdmrt_oracle.so")
SRC_PATH = os.path.join(_HERE, "dmrt_oracle.c")

CAVITY, PERIODIC, CHANNEL_X, ADIABATIC_BOX = 0, 1, 2, 3
Q5_FIXED_A, Q5_PAPER = 0, 1
MRT, LBGK = 0, 1
OK, EINVAL, EUNSTABLE, ENOMEM = 0, -1, -2, -3

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, IEEE double, no fast-math)."""
    if force or not os.path.exists(LIB_PATH) or (
            os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH)):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fno-fast-math",
                               "-ffp-contract=off", "-shared", "-fPIC",
                               SRC_PATH, "-o", tmp, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        L.orc_derive.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                 _dp]
        L.orc_derive.restype = ctypes.c_int
        L.orc_create.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_int, _ip]
        L.orc_create.restype = ctypes.c_void_p
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_destroy.restype = None
        for name, args in [
            ("orc_derived", [ctypes.c_void_p, _dp]),
            ("orc_matrices", [ctypes.c_void_p, _dp, _dp, _dp, _dp, _ip, _ip]),
            ("orc_force", [ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                           ctypes.c_double, ctypes.c_double, _dp]),
            ("orc_collide", [ctypes.c_void_p, _dp, _dp, _dp, _dp]),
            ("orc_set_rates", [ctypes.c_void_p, _dp, _dp]),
            ("orc_set_equilibrium", [ctypes.c_void_p, _dp, _dp, _dp, _dp]),
            ("orc_set_hot_wall", [ctypes.c_void_p, _dp]),
            ("orc_get_state", [ctypes.c_void_p, _dp, _dp]),
            ("orc_set_state", [ctypes.c_void_p, _dp, _dp]),
            ("orc_step", [ctypes.c_void_p, ctypes.c_long]),
            ("orc_fields", [ctypes.c_void_p, _dp, _dp, _dp, _dp]),
            ("orc_nusselt", [ctypes.c_void_p, ctypes.c_int, _dp, _dp]),
        ]:
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.orc_objective.argtypes = [ctypes.c_void_p, ctypes.c_long, ctypes.c_long, _dp]
        L.orc_objective.restype = ctypes.c_int
        L.orc_steps.argtypes = [ctypes.c_void_p]
        L.orc_steps.restype = ctypes.c_long
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle error {code}")
        self.code = code


def _check(rc):
    if rc != OK:
        raise OracleError(rc)


DERIVED_KEYS = ("nu", "alpha", "gbeta", "s_nu", "s_q", "sigma_k", "sigma_e",
                "sigma_nu", "a", "w0", "wm", "H")


def derive(n, Ra, Pr, Ma, theta_hot=0.5, theta_cold=-0.5, q5_mode=Q5_FIXED_A,
           a=-2.0 / 3.0, gbeta_override=math.nan, collision=MRT):
    out = np.zeros(12)
    _check(lib().orc_derive(n, Ra, Pr, Ma, theta_hot, theta_cold, q5_mode, a,
                            gbeta_override, collision, _ptr(out)))
    return dict(zip(DERIVED_KEYS, out.tolist()))


class Oracle:
    """One square cavity (or periodic / channel / adiabatic test box)."""

    def __init__(self, n, Ra, Pr, Ma=0.1, theta_hot=0.5, theta_cold=-0.5,
                 q5_mode=Q5_FIXED_A, a=-2.0 / 3.0, bc=CAVITY,
                 gbeta_override=math.nan, force_x=0.0, theta_ref=0.0, collision=MRT):
        err = ctypes.c_int(0)
        h = lib().orc_create(n, Ra, Pr, Ma, theta_hot, theta_cold, q5_mode, a, bc,
                             gbeta_override, force_x, theta_ref, collision, ctypes.byref(err))
        if not h:
            raise OracleError(err.value)
        self._h = h
        self.n = n
        self.theta_hot, self.theta_cold = theta_hot, theta_cold

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    # -- parameters and matrices ------------------------------------------
    def derived(self):
        out = np.zeros(18)
        _check(lib().orc_derived(self._h, _ptr(out)))
        return {"nu": out[0], "alpha": out[1], "gbeta": out[2],
                "S": out[3:12].copy(), "Q": out[12:17].copy(), "a": out[17]}

    def matrices(self):
        M = np.zeros(81); Mi = np.zeros(81); N = np.zeros(25); Ni = np.zeros(25)
        e9 = np.zeros(18, dtype=np.int32); e5 = np.zeros(10, dtype=np.int32)
        _check(lib().orc_matrices(self._h, _ptr(M), _ptr(Mi), _ptr(N), _ptr(Ni),
                                  e9.ctypes.data_as(_ip), e5.ctypes.data_as(_ip)))
        return (M.reshape(9, 9), Mi.reshape(9, 9), N.reshape(5, 5), Ni.reshape(5, 5),
                e9.reshape(9, 2), e5.reshape(5, 2))

    # -- single node --------------------------------------------------------
    def collide(self, f, g):
        f = np.ascontiguousarray(f, dtype=np.float64)
        g = np.ascontiguousarray(g, dtype=np.float64)
        fs = np.zeros(9); gs = np.zeros(5)
        _check(lib().orc_collide(self._h, _ptr(f), _ptr(g), _ptr(fs), _ptr(gs)))
        return fs, gs

    def set_rates(self, S, Q):
        """Test hook: overwrite the relaxation rates of Eqs. 31 and 38."""
        S = np.ascontiguousarray(S, dtype=np.float64).reshape(9)
        Q = np.ascontiguousarray(Q, dtype=np.float64).reshape(5)
        _check(lib().orc_set_rates(self._h, _ptr(S), _ptr(Q)))

    def force(self, Gx, Gy, u, v):
        F = np.zeros(9)
        _check(lib().orc_force(self._h, Gx, Gy, u, v, _ptr(F)))
        return F

    # -- state ----------------------------------------------------------------
    def set_equilibrium(self, drho=None, U=None, V=None, theta=None):
        nn = self.n * self.n
        conv = [None if a is None else np.ascontiguousarray(
            np.broadcast_to(np.asarray(a, dtype=np.float64), (self.n, self.n))
        ).reshape(nn) for a in (drho, U, V, theta)]
        _check(lib().orc_set_equilibrium(self._h, *[_ptr(a) for a in conv]))

    def set_theta(self, theta0):
        self.set_equilibrium(theta=theta0)

    def set_hot_wall(self, theta_w):
        tw = np.ascontiguousarray(theta_w, dtype=np.float64).reshape(self.n)
        _check(lib().orc_set_hot_wall(self._h, _ptr(tw)))

    def get_state(self):
        nn = self.n * self.n
        f = np.zeros(nn * 9); g = np.zeros(nn * 5)
        _check(lib().orc_get_state(self._h, _ptr(f), _ptr(g)))
        return f.reshape(self.n, self.n, 9), g.reshape(self.n, self.n, 5)

    def set_state(self, f, g):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        g = np.ascontiguousarray(g, dtype=np.float64).reshape(-1)
        assert f.size == self.n * self.n * 9 and g.size == self.n * self.n * 5
        _check(lib().orc_set_state(self._h, _ptr(f), _ptr(g)))

    def step(self, nsteps=1):
        _check(lib().orc_step(self._h, int(nsteps)))

    @property
    def steps(self):
        return lib().orc_steps(self._h)

    def objective(self, nsteps, avg_last):
        """Step nsteps and return the mean hot-wall Nu_avg over the last
        avg_last steps."""
        J = ctypes.c_double(0.0)
        _check(lib().orc_objective(self._h, int(nsteps), int(avg_last), ctypes.byref(J)))
        return J.value

    # -- diagnostics ----------------------------------------------------------
    def fields(self):
        """Return U, V, theta, P as (n, n) arrays indexed [y, x]."""
        nn = self.n * self.n
        U = np.zeros(nn); V = np.zeros(nn); T = np.zeros(nn); P = np.zeros(nn)
        _check(lib().orc_fields(self._h, _ptr(U), _ptr(V), _ptr(T), _ptr(P)))
        s = (self.n, self.n)
        return U.reshape(s), V.reshape(s), T.reshape(s), P.reshape(s)

    def nusselt(self, wall=0):
        loc = np.zeros(self.n)
        avg = ctypes.c_double(0.0)
        _check(lib().orc_nusselt(self._h, wall, ctypes.byref(avg), _ptr(loc)))
        return avg.value, loc
