"""Thin ctypes binding of libdmrt (include/dmrt.h): argument marshalling only.

Every function here has the name of the C entry point it wraps and returns
its integer code; ``check`` turns a code into an exception.  All compute runs
in the library's HIP kernels.  If libdmrt.so has not been built, importing
this module raises: there is no fallback path.

``Cavity`` is a convenience owner of one ``dmrt_cavity*`` handle that
allocates numpy outputs and raises ``DmrtError`` on failure.  Optionally its
distribution buffers and stream come from PyTorch (device memory and stream
plumbing only).
"""
from __future__ import annotations

import ctypes
import math
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# DMRT_LIB: path of another build of the same library (e.g. a variant under test)
LIB_PATH = os.environ.get("DMRT_LIB") or os.path.join(_HERE, "libdmrt.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "dmrt.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
        "(or python paper_1601_04633_amd/build.py); there is no CPU fallback")

# One HIP runtime per process.  PyTorch ships its own libamdhip64.so.7 and
# looks it up under another file name, so if libdmrt loaded the system copy
# first, torch would load a second runtime that cannot open the GPU.  Loading
# torch first makes libdmrt bind to the runtime torch already mapped.
try:
    import torch  # noqa: F401
except ImportError:  # pure C-ABI use without PyTorch
    torch = None

_lib = ctypes.CDLL(LIB_PATH)


def _header_defines():
    vals = {}
    with open(HEADER_PATH) as fh:
        for line in fh:
            m = re.match(r"#define\s+(DMRT_\w+)\s+(-?\d+)", line)
            if m:
                vals[m.group(1)] = int(m.group(2))
    return vals


globals().update(_header_defines())


class dmrt_params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int),
                ("Ra", ctypes.c_double), ("Pr", ctypes.c_double), ("Ma", ctypes.c_double),
                ("theta_hot", ctypes.c_double), ("theta_cold", ctypes.c_double),
                ("precision", ctypes.c_int), ("q5_mode", ctypes.c_int), ("a", ctypes.c_double),
                ("bc_mode", ctypes.c_int), ("gbeta_override", ctypes.c_double),
                ("force_x", ctypes.c_double), ("theta_ref", ctypes.c_double),
                ("collision", ctypes.c_int)]


class dmrt_derived(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in
                ("nu", "alpha", "gbeta", "s_nu", "s_q", "sigma_k", "sigma_e", "sigma_nu",
                 "a", "w0", "wm", "H")]


_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_P = ctypes.POINTER(dmrt_params)
_c_int, _c_long, _c_size = ctypes.c_int, ctypes.c_long, ctypes.c_size_t

_SIGS = {
    "dmrt_params_default": [_P],
    "dmrt_derive": [_P, ctypes.POINTER(dmrt_derived)],
    "dmrt_buffer_bytes": [_P, ctypes.POINTER(_c_size), ctypes.POINTER(_c_size)],
    "dmrt_create": [_P, _vp, _vp, _vp, ctypes.POINTER(_vp)],
    "dmrt_set_theta": [_vp, _dp],
    "dmrt_set_equilibrium": [_vp, _dp, _dp, _dp, _dp],
    "dmrt_set_hot_wall": [_vp, _dp],
    "dmrt_step": [_vp, _c_long],
    "dmrt_sync": [_vp],
    "dmrt_get_step": [_vp, ctypes.POINTER(_c_long)],
    "dmrt_get_fields": [_vp, _dp, _dp, _dp, _dp],
    "dmrt_nusselt": [_vp, _c_int, _dp, _dp],
    "dmrt_nu_series": [_vp, _c_int, _c_long],
    "dmrt_nu_series_read": [_vp, _dp, ctypes.POINTER(_c_long)],
    "dmrt_residual": [_vp, _dp, _dp],
    "dmrt_residual_noalloc": [_vp, _vp, _dp, _dp],
    "dmrt_state_bytes": [_vp, ctypes.POINTER(_c_size)],
    "dmrt_save_state": [_vp, _vp, _c_size],
    "dmrt_load_state": [_vp, _vp, _c_size],
    "dmrt_set_launch": [_vp, _c_int, _c_int, _c_int, _c_int],
    "dmrt_set_temporal": [_vp, _c_int, _c_int],
    "dmrt_set_temporal_march": [_vp, _c_int, _c_int, _c_int],
    "dmrt_get_temporal_march": [_vp, ctypes.POINTER(_c_int), ctypes.POINTER(_c_int)],
    "dmrt_buffers": [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_c_int)],
    "dmrt_destroy": [_vp],
    "dmrt_adjoint_forward": [_vp, _c_long, _c_long, _c_long, _dp],
    "dmrt_adjoint_backward": [_vp, _dp, _dp],
    "dmrt_adjoint_nu": [_vp, _c_long, _c_long, _c_long, _dp, _dp, _dp],
    "dmrt_adjoint_release": [_vp],
    "dmrt_adjoint_generation": [_vp, ctypes.POINTER(_c_long)],
    "dmrt_adjoint_set_temporal": [_vp, _c_int, _c_int],
    "dmrt_batch_create": [_P, _c_int, _vp, ctypes.POINTER(_vp)],
    "dmrt_batch_set_theta": [_vp, _c_int, _dp],
    "dmrt_batch_set_hot_wall": [_vp, _c_int, _dp],
    "dmrt_batch_set_schedule": [_vp, _c_int, _c_int, _c_int, _c_int, _c_size, _c_int],
    "dmrt_batch_set_temporal": [_vp, _c_int, _c_int],
    "dmrt_batch_set_temporal_march": [_vp, _c_int, _c_int, _c_int],
    "dmrt_batch_step": [_vp, _c_long],
    "dmrt_batch_sync": [_vp],
    "dmrt_batch_get_step": [_vp, ctypes.POINTER(_c_long)],
    "dmrt_batch_nusselt": [_vp, _dp],
    "dmrt_batch_status": [_vp, ctypes.POINTER(_c_int)],
    "dmrt_batch_get_fields": [_vp, _c_int, _dp, _dp, _dp, _dp],
    "dmrt_batch_member_state": [_vp, _c_int, _vp, _vp],
    "dmrt_batch_load_member_state": [_vp, _c_int, _vp, _vp],
    "dmrt_batch_destroy": [_vp],
}

for _name, _args in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = ctypes.c_int
    globals()[_name] = _fn

_lib.dmrt_strerror.argtypes = [ctypes.c_int]
_lib.dmrt_strerror.restype = ctypes.c_char_p
_lib.dmrt_last_error.argtypes = []
_lib.dmrt_last_error.restype = ctypes.c_char_p


def dmrt_strerror(code: int) -> str:
    return _lib.dmrt_strerror(code).decode()


def dmrt_last_error() -> str:
    return _lib.dmrt_last_error().decode()


class DmrtError(RuntimeError):
    def __init__(self, code, where=""):
        detail = dmrt_last_error() if code == DMRT_EHIP else ""
        super().__init__(f"{where}: {dmrt_strerror(code)} ({code}) {detail}".strip())
        self.code = code


def check(code: int, where: str = "") -> None:
    if code != DMRT_OK:
        raise DmrtError(code, where)


def exported_symbols():
    """Names of the functions declared in include/dmrt.h."""
    text = open(HEADER_PATH).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+char\s*\*|int)\s*(dmrt_\w+)\s*\(", text,
                                 flags=re.M)))


def make_params(n=64, Ra=1e3, Pr=0.01, Ma=0.1, theta_hot=0.5, theta_cold=-0.5,
                precision="fp64", q5_mode=None, a=-2.0 / 3.0, bc_mode=None,
                gbeta_override=math.nan, force_x=0.0, theta_ref=0.0,
                collision=None) -> dmrt_params:
    p = dmrt_params()
    check(dmrt_params_default(ctypes.byref(p)), "dmrt_params_default")
    p.n, p.Ra, p.Pr, p.Ma = n, Ra, Pr, Ma
    p.theta_hot, p.theta_cold = theta_hot, theta_cold
    p.precision = {"fp32": DMRT_FP32, "fp64": DMRT_FP64}[precision] \
        if isinstance(precision, str) else int(precision)
    p.q5_mode = DMRT_Q5_FIXED_A if q5_mode is None else q5_mode
    p.a = a
    p.bc_mode = DMRT_BC_CAVITY if bc_mode is None else bc_mode
    p.gbeta_override, p.force_x, p.theta_ref = gbeta_override, force_x, theta_ref
    if isinstance(collision, str):
        collision = {"mrt": DMRT_COLL_MRT, "lbgk": DMRT_COLL_LBGK}[collision.lower()]
    p.collision = DMRT_COLL_MRT if collision is None else int(collision)
    return p


def derive(p: dmrt_params) -> dict:
    d = dmrt_derived()
    check(dmrt_derive(ctypes.byref(p), ctypes.byref(d)), "dmrt_derive")
    return {k: getattr(d, k) for k, _ in dmrt_derived._fields_}


def _arr(a, size):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
    if a.size != size:
        raise ValueError(f"expected {size} values, got {a.size}")
    return a


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


class Cavity:
    """One cavity handle.  ``torch_buffers=True`` allocates the distribution
    buffers as torch CUDA tensors and enqueues on torch's current stream."""

    def __init__(self, torch_buffers: bool = False, stream=None, **kw):
        self.params = make_params(**kw)
        self.n = self.params.n
        self._tensors = None
        ext_f = ext_g = None
        if torch_buffers:
            import torch
            fb, gb = ctypes.c_size_t(0), ctypes.c_size_t(0)
            check(dmrt_buffer_bytes(ctypes.byref(self.params), ctypes.byref(fb), ctypes.byref(gb)),
                  "dmrt_buffer_bytes")
            tf = torch.empty(fb.value, dtype=torch.uint8, device="cuda")
            tg = torch.empty(gb.value, dtype=torch.uint8, device="cuda")
            self._tensors = (tf, tg)
            ext_f, ext_g = tf.data_ptr(), tg.data_ptr()
            if stream is None:
                stream = torch.cuda.current_stream().cuda_stream or None
        h = ctypes.c_void_p()
        check(dmrt_create(ctypes.byref(self.params), ext_f, ext_g, stream, ctypes.byref(h)),
              "dmrt_create")
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            dmrt_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def derived(self):
        return derive(self.params)

    def set_theta(self, theta0):
        check(dmrt_set_theta(self._h, _ptr(_arr(theta0, self.n * self.n))), "dmrt_set_theta")

    def set_equilibrium(self, drho=None, U=None, V=None, theta=None):
        nn = self.n * self.n
        arrs = [None if a is None else _arr(np.broadcast_to(np.asarray(a, dtype=np.float64),
                                                            (self.n, self.n)), nn)
                for a in (drho, U, V, theta)]
        check(dmrt_set_equilibrium(self._h, *[_ptr(a) for a in arrs]), "dmrt_set_equilibrium")

    def set_hot_wall(self, theta_w):
        check(dmrt_set_hot_wall(self._h, _ptr(_arr(theta_w, self.n))), "dmrt_set_hot_wall")

    def step(self, nsteps=1):
        check(dmrt_step(self._h, int(nsteps)), "dmrt_step")

    def sync(self):
        check(dmrt_sync(self._h), "dmrt_sync")

    @property
    def steps(self):
        s = ctypes.c_long(0)
        check(dmrt_get_step(self._h, ctypes.byref(s)), "dmrt_get_step")
        return s.value

    def fields(self):
        """U, V, theta, P as (n, n) arrays indexed [y, x]."""
        nn = self.n * self.n
        out = [np.empty(nn) for _ in range(4)]
        check(dmrt_get_fields(self._h, *[_ptr(a) for a in out]), "dmrt_get_fields")
        return tuple(a.reshape(self.n, self.n) for a in out)

    def nusselt(self, wall=0):
        avg = ctypes.c_double(0.0)
        loc = np.empty(self.n)
        check(dmrt_nusselt(self._h, wall, ctypes.byref(avg), _ptr(loc)), "dmrt_nusselt")
        return avg.value, loc

    def nu_series(self, stride, cap):
        check(dmrt_nu_series(self._h, int(stride), int(cap)), "dmrt_nu_series")
        self._ring_cap = int(cap)

    def nu_series_read(self):
        cap = getattr(self, "_ring_cap", 0)
        out = np.empty(max(cap, 1))
        cnt = ctypes.c_long(0)
        check(dmrt_nu_series_read(self._h, _ptr(out), ctypes.byref(cnt)), "dmrt_nu_series_read")
        return out[:cnt.value].copy()

    def residual(self):
        rt, ru = ctypes.c_double(0), ctypes.c_double(0)
        rc = dmrt_residual(self._h, ctypes.byref(rt), ctypes.byref(ru))
        if rc not in (DMRT_OK, DMRT_ENONFINITE):
            check(rc, "dmrt_residual")
        return rt.value, ru.value, rc == DMRT_ENONFINITE

    def residual_noalloc(self, ref_ptr):
        """dmrt_residual_noalloc with the reference fields at device address
        ref_ptr (3 n^2 doubles, caller-owned)."""
        rt, ru = ctypes.c_double(0), ctypes.c_double(0)
        rc = dmrt_residual_noalloc(self._h, ref_ptr, ctypes.byref(rt), ctypes.byref(ru))
        if rc not in (DMRT_OK, DMRT_ENONFINITE):
            check(rc, "dmrt_residual_noalloc")
        return rt.value, ru.value, rc == DMRT_ENONFINITE

    def save_state(self) -> bytes:
        nb = ctypes.c_size_t(0)
        check(dmrt_state_bytes(self._h, ctypes.byref(nb)), "dmrt_state_bytes")
        buf = ctypes.create_string_buffer(nb.value)
        check(dmrt_save_state(self._h, buf, nb.value), "dmrt_save_state")
        return buf.raw

    def load_state(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        check(dmrt_load_state(self._h, buf, len(blob)), "dmrt_load_state")

    def set_launch(self, block_x=256, block_y=1, xcd_remap=1, graph_steps=64):
        check(dmrt_set_launch(self._h, block_x, block_y, xcd_remap, graph_steps), "dmrt_set_launch")

    # -- gradient of the time-averaged hot-wall Nusselt number ------------------
    def adjoint_forward(self, nsteps, avg_last, ckpt_every=500):
        J = ctypes.c_double(0.0)
        check(dmrt_adjoint_forward(self._h, int(nsteps), int(avg_last), int(ckpt_every),
                                   ctypes.byref(J)), "dmrt_adjoint_forward")
        return J.value

    def adjoint_backward(self):
        gw = np.empty(self.n)
        g0 = np.empty(self.n * self.n)
        check(dmrt_adjoint_backward(self._h, _ptr(gw), _ptr(g0)), "dmrt_adjoint_backward")
        return gw, g0.reshape(self.n, self.n)

    def adjoint_nu(self, nsteps, avg_last, ckpt_every=500):
        J = ctypes.c_double(0.0)
        gw = np.empty(self.n)
        g0 = np.empty(self.n * self.n)
        check(dmrt_adjoint_nu(self._h, int(nsteps), int(avg_last), int(ckpt_every), ctypes.byref(J),
                              _ptr(gw), _ptr(g0)), "dmrt_adjoint_nu")
        return J.value, gw, g0.reshape(self.n, self.n)

    def adjoint_generation(self):
        """Generation of the stored forward run (0: none usable)."""
        g = ctypes.c_long(0)
        check(dmrt_adjoint_generation(self._h, ctypes.byref(g)), "dmrt_adjoint_generation")
        return g.value

    def adjoint_release(self):
        check(dmrt_adjoint_release(self._h), "dmrt_adjoint_release")

    def adjoint_set_temporal(self, steps_per_launch=4, tile_rows=16):
        check(dmrt_adjoint_set_temporal(self._h, steps_per_launch, tile_rows),
              "dmrt_adjoint_set_temporal")

    def set_temporal(self, steps_per_launch=4, tile_rows=16):
        check(dmrt_set_temporal(self._h, steps_per_launch, tile_rows), "dmrt_set_temporal")

    def set_temporal_march(self, steps_per_launch=4, group_rows=4, chunk_rows=0):
        """K steps per launch with workgroups marching up chunks of rows;
        returns the rows per workgroup in use."""
        check(dmrt_set_temporal_march(self._h, steps_per_launch, group_rows, chunk_rows),
              "dmrt_set_temporal_march")
        return self.temporal_march()[1]

    def temporal_march(self):
        """(wave rows per step group, rows per workgroup); (0, 0) when off."""
        b, c = _c_int(0), _c_int(0)
        check(dmrt_get_temporal_march(self._h, ctypes.byref(b), ctypes.byref(c)),
              "dmrt_get_temporal_march")
        return b.value, c.value

    def buffers(self):
        f, g, c = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_int(0)
        check(dmrt_buffers(self._h, ctypes.byref(f), ctypes.byref(g), ctypes.byref(c)), "dmrt_buffers")
        return f.value, g.value, c.value

    def raw_state(self):
        """Post-collision state of the current step as (f[9, n, n], g[5, n, n])
        in the storage precision (from a checkpoint blob)."""
        blob = self.save_state()
        n = self.n
        dt = np.float64 if self.params.precision == DMRT_FP64 else np.float32
        off = 8 * 8 + n * 8
        data = np.frombuffer(blob, dtype=dt, offset=off, count=14 * n * n)
        return data[:9 * n * n].reshape(9, n, n).copy(), data[9 * n * n:].reshape(5, n, n).copy()


class Batch:
    """A batched sweep of independent cavities (one launch per step).

    ``members``: list of dicts of ``make_params`` keywords (n, Ra, Pr, ...),
    all with the same precision."""

    def __init__(self, members, precision="fp32", stream=None):
        self.members = [dict(m) for m in members]
        arr = (dmrt_params * len(members))()
        for i, m in enumerate(self.members):
            kw = dict(m)
            kw.setdefault("precision", precision)
            arr[i] = make_params(**kw)
        self.params = arr
        self.count = len(members)
        self.precision = arr[0].precision
        h = ctypes.c_void_p()
        check(dmrt_batch_create(arr, self.count, stream, ctypes.byref(h)), "dmrt_batch_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            dmrt_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def n(self, i):
        return self.params[i].n

    def set_theta(self, i, theta0):
        check(dmrt_batch_set_theta(self._h, i, _ptr(_arr(theta0, self.n(i) ** 2))),
              "dmrt_batch_set_theta")

    def set_hot_wall(self, i, theta_w):
        check(dmrt_batch_set_hot_wall(self._h, i, _ptr(_arr(theta_w, self.n(i)))),
              "dmrt_batch_set_hot_wall")

    def set_schedule(self, block_x=64, block_y=4, order=1, grid_blocks=0, group_bytes=0,
                     group_steps=64):
        check(dmrt_batch_set_schedule(self._h, block_x, block_y, order, grid_blocks,
                                      int(group_bytes), group_steps), "dmrt_batch_set_schedule")

    def set_temporal(self, steps_per_launch=4, tile_rows=16):
        check(dmrt_batch_set_temporal(self._h, steps_per_launch, tile_rows), "dmrt_batch_set_temporal")

    def set_temporal_march(self, steps_per_launch=4, group_rows=3, chunk_rows=0):
        """K steps per launch with the row-marching sweep (one member's
        column band and chunk of rows per workgroup)."""
        check(dmrt_batch_set_temporal_march(self._h, steps_per_launch, group_rows, chunk_rows),
              "dmrt_batch_set_temporal_march")

    def step(self, nsteps=1):
        check(dmrt_batch_step(self._h, int(nsteps)), "dmrt_batch_step")

    def sync(self):
        check(dmrt_batch_sync(self._h), "dmrt_batch_sync")

    @property
    def steps(self):
        s = ctypes.c_long(0)
        check(dmrt_batch_get_step(self._h, ctypes.byref(s)), "dmrt_batch_get_step")
        return s.value

    def nusselt(self):
        out = np.empty(self.count)
        check(dmrt_batch_nusselt(self._h, _ptr(out)), "dmrt_batch_nusselt")
        return out

    def status(self):
        out = (ctypes.c_int * self.count)()
        check(dmrt_batch_status(self._h, out), "dmrt_batch_status")
        return np.array(list(out))

    def fields(self, i):
        n = self.n(i)
        out = [np.empty(n * n) for _ in range(4)]
        check(dmrt_batch_get_fields(self._h, i, *[_ptr(a) for a in out]), "dmrt_batch_get_fields")
        return tuple(a.reshape(n, n) for a in out)

    def raw_state(self, i):
        n = self.n(i)
        dt = np.float64 if self.precision == DMRT_FP64 else np.float32
        f = np.empty((9, n, n), dtype=dt)
        g = np.empty((5, n, n), dtype=dt)
        check(dmrt_batch_member_state(self._h, i, f.ctypes.data, g.ctypes.data),
              "dmrt_batch_member_state")
        return f, g

    def load_state(self, i, f, g):
        dt = np.float64 if self.precision == DMRT_FP64 else np.float32
        n = self.n(i)
        f = np.ascontiguousarray(f, dtype=dt).reshape(9, n, n)
        g = np.ascontiguousarray(g, dtype=dt).reshape(5, n, n)
        check(dmrt_batch_load_member_state(self._h, i, f.ctypes.data, g.ctypes.data),
              "dmrt_batch_load_member_state")
