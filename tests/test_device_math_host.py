"""CPU pins of the device arithmetic itself: the collision and its
vector-Jacobian product from the kernels' header, compiled for the host
(tests/host_math), against the oracle's collision (FP64) and against
central differences of that same collision.  No GPU needed."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def host_lib():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out_dir = os.path.join(HERE, "host_math", "_build")
    os.makedirs(out_dir, exist_ok=True)
    so = os.path.join(out_dir, "device_math_host.so")
    subprocess.run([hipcc, "--offload-host-only", "-std=c++17", "-O1", "-fPIC", "-shared",
                    "-I" + os.path.join(ROOT, "include"),
                    "-I" + os.path.join(ROOT, "paper_1601_04633_amd", "csrc"),
                    os.path.join(HERE, "host_math", "device_math_host.hip"), "-o", so],
                   check=True, capture_output=True)
    lib = ctypes.CDLL(so)
    dp = ctypes.POINTER(ctypes.c_double)
    for name in ("dmrt_host_collide", "dmrt_host_collide_vjp"):
        getattr(lib, name).argtypes = [ctypes.c_void_p, ctypes.c_void_p, dp, dp, dp, dp]
        getattr(lib, name).restype = ctypes.c_int
    fp = ctypes.POINTER(ctypes.c_float)
    for name, ptr in (("dmrt_host_vjp_paths_f64", dp), ("dmrt_host_vjp_paths_f32", fp)):
        getattr(lib, name).argtypes = [ctypes.c_void_p, ctypes.c_void_p, ptr, ptr, ptr, ptr, ptr]
        getattr(lib, name).restype = ctypes.c_int
    return lib


def _params(bc_mode=0, **kw):
    from paper_1601_04633_amd import dmrt as D
    p = D.make_params(precision=1, bc_mode=bc_mode, **kw)
    d = D.dmrt_derived()
    assert D.dmrt_derive(ctypes.byref(p), ctypes.byref(d)) == 0
    return p, d


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _collide(lib, p, d, f, g):
    f = np.ascontiguousarray(f, dtype=np.float64).copy()
    g = np.ascontiguousarray(g, dtype=np.float64).copy()
    fs, gs = np.zeros(9), np.zeros(5)
    lib.dmrt_host_collide(ctypes.byref(p), ctypes.byref(d), _p(f), _p(g), _p(fs), _p(gs))
    return fs, gs


def _states(rng, count, scale_f=0.05, scale_g=0.3):
    for _ in range(count):
        yield rng.uniform(-scale_f, scale_f, 9), rng.uniform(-scale_g, scale_g, 5)


# cavity (no horizontal force) and the test modes (horizontal force, other
# buoyancy and reference temperature), large forcing so every force term counts
CASES = [
    dict(bc_mode=0, n=64, Ra=1e4, Pr=0.01),
    dict(bc_mode=0, n=32, Ra=1e5, Pr=0.001, gbeta_override=0.3, theta_ref=0.1),
    dict(bc_mode=1, n=48, Ra=3e3, Pr=0.05, gbeta_override=0.2, force_x=0.05),
    dict(bc_mode=2, n=40, Ra=1e3, Pr=0.1, gbeta_override=0.0, force_x=0.1),
    # double LBGK: the device's moment-space collision with equal rates
    # against the oracle's distribution-space BGK
    dict(bc_mode=0, n=256, Ra=5e4, Pr=0.005, collision=1),
    dict(bc_mode=1, n=48, Ra=3e3, Pr=0.05, gbeta_override=0.2, force_x=0.05, collision=1),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_device_collision_matches_oracle(host_lib, oracle_mod, case):
    kw = dict(CASES[case])
    p, d = _params(**kw)
    okw = {k: v for k, v in kw.items() if k not in ("bc_mode", "n", "Ra", "Pr")}
    o = oracle_mod.Oracle(kw["n"], kw["Ra"], kw["Pr"], bc=kw["bc_mode"], **okw)
    rng = np.random.default_rng(100 + case)
    for f, g in _states(rng, 200):
        fs, gs = _collide(host_lib, p, d, f, g)
        fo, go = o.collide(f, g)
        assert np.abs(fs - fo).max() <= 2e-15 * max(1.0, np.abs(fo).max()), (fs - fo)
        assert np.abs(gs - go).max() <= 2e-15 * max(1.0, np.abs(go).max()), (gs - go)


@pytest.mark.parametrize("case", [0, 1])
def test_collision_vjp_matches_central_differences(host_lib, case):
    kw = dict(CASES[case])
    p, d = _params(**kw)
    rng = np.random.default_rng(200 + case)
    h = 1e-6
    for f, g in _states(rng, 100):
        lf, lg = rng.standard_normal(9), rng.standard_normal(5)
        df, dg = rng.standard_normal(9), rng.standard_normal(5)
        fp, gp = _collide(host_lib, p, d, f + h * df, g + h * dg)
        fm, gm = _collide(host_lib, p, d, f - h * df, g - h * dg)
        fd = (lf @ (fp - fm) + lg @ (gp - gm)) / (2 * h)
        a, b = lf.copy(), lg.copy()
        host_lib.dmrt_host_collide_vjp(ctypes.byref(p), ctypes.byref(d), _p(f.copy()), _p(g.copy()),
                                       _p(a), _p(b))
        ad = a @ df + b @ dg
        assert abs(ad - fd) <= 1e-8 * max(1.0, abs(fd)), (ad, fd)


def test_collision_vjp_is_exact_for_the_linear_part(host_lib):
    """At rest with theta = 0 and no buoyancy, the collision is linear in
    small perturbations about the state to first order; the VJP must then
    be the transpose of the finite-difference Jacobian column by column."""
    p, d = _params(bc_mode=0, n=64, Ra=1e4, Pr=0.01, gbeta_override=0.0)
    f0, g0 = np.zeros(9), np.zeros(5)
    h = 1e-7
    J = np.zeros((14, 14))
    for k in range(14):
        e = np.zeros(14); e[k] = h
        fp, gp = _collide(host_lib, p, d, f0 + e[:9], g0 + e[9:])
        fm, gm = _collide(host_lib, p, d, f0 - e[:9], g0 - e[9:])
        J[:, k] = np.concatenate([fp - fm, gp - gm]) / (2 * h)
    for r in range(14):
        lam = np.zeros(14); lam[r] = 1.0
        a, b = lam[:9].copy(), lam[9:].copy()
        host_lib.dmrt_host_collide_vjp(ctypes.byref(p), ctypes.byref(d), _p(f0.copy()), _p(g0.copy()),
                                       _p(a), _p(b))
        assert np.abs(np.concatenate([a, b]) - J[r]).max() <= 1e-8


def test_collision_vjp_dot_product_identity(host_lib):
    """<J v, w> = <v, J^T w> for the collision at random states, with J v
    from forward-mode differentiation of the vectorised FP64 reference
    (oracle/torch_ref.py, matrix form with M^-1, N^-1) and J^T w from the
    device's hand-derived VJP: equal to round-off (1e-13)."""
    torch = pytest.importorskip("torch")
    from oracle.torch_ref import Reference
    n, Ra, Pr = 64, 1e4, 0.01
    ref = Reference(n, Ra, Pr)
    p, d = _params(bc_mode=0, n=n, Ra=Ra, Pr=Pr)
    rng = np.random.default_rng(17)
    m = 64
    f = rng.uniform(-0.05, 0.05, (9, 1, m))
    g = rng.uniform(-0.4, 0.4, (5, 1, m))
    vf, vg = rng.standard_normal((9, 1, m)), rng.standard_normal((5, 1, m))
    wf, wg = rng.standard_normal((9, 1, m)), rng.standard_normal((5, 1, m))
    _, (jf, jg) = torch.func.jvp(ref.collide, (torch.tensor(f), torch.tensor(g)),
                                 (torch.tensor(vf), torch.tensor(vg)))
    lhs = (jf.numpy() * wf).sum(axis=0)[0] + (jg.numpy() * wg).sum(axis=0)[0]
    for k in range(m):
        a, b = wf[:, 0, k].copy(), wg[:, 0, k].copy()
        host_lib.dmrt_host_collide_vjp(ctypes.byref(p), ctypes.byref(d), _p(f[:, 0, k].copy()),
                                       _p(g[:, 0, k].copy()), _p(a), _p(b))
        rhs = a @ vf[:, 0, k] + b @ vg[:, 0, k]
        scale = np.abs(wf[:, 0, k]).sum() + np.abs(wg[:, 0, k]).sum()
        assert abs(lhs[k] - rhs) <= 1e-13 * scale, (k, lhs[k], rhs)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_vjp_at_forward_point_is_bitwise_the_state_vjp(host_lib, dtype):
    """The backward stores only the u, v, theta that the forward collision
    returns and forms the transposed Jacobian from them: that must be
    bitwise the transposed Jacobian formed from the whole pre-collision
    state (the Jacobian depends on the state only through u, v, theta), in
    both storage precisions, for states across the moment ranges of the
    cavity runs (including walls' extreme temperatures)."""
    p, d = _params(Ra=1e4, Pr=0.01, n=256)
    rng = np.random.default_rng(4633)
    name = "dmrt_host_vjp_paths_f64" if dtype == np.float64 else "dmrt_host_vjp_paths_f32"
    ct = ctypes.c_double if dtype == np.float64 else ctypes.c_float
    fn = getattr(host_lib, name)

    def ptr(a):
        return a.ctypes.data_as(ctypes.POINTER(ct))

    count = 0
    for scale_f, scale_g in ((1e-6, 1e-4), (0.05, 0.3), (0.2, 0.6)):
        for f, g in _states(rng, 200, scale_f, scale_g):
            f = f.astype(dtype)
            g = g.astype(dtype)
            lam = rng.normal(size=14).astype(dtype)
            a = np.zeros(14, dtype)
            b = np.zeros(14, dtype)
            fn(ctypes.byref(p), ctypes.byref(d), ptr(f), ptr(g), ptr(lam), ptr(a), ptr(b))
            assert np.isfinite(a).all()
            assert a.tobytes() == b.tobytes(), (f, g, lam, a, b)
            count += 1
    assert count == 600
