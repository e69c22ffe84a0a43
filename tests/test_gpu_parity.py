"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on
the same seeded inputs.

Bars (field-norm relative error ||x_gpu - x_ref||_2 / ||x_ref||_2 per field):
  FP64 GPU vs oracle                 <= 1e-12 on U, V, theta, P and Nu
  FP32 GPU vs oracle / FP64 GPU      <= 1e-5 on U, V, theta; <= 1e-4 on Nu
Sizes span several 256-wide tiles and ragged tails (n not a multiple of 64),
the smallest grid (n = 4), every wall configuration, and the full 1024^2
configuration in the launch shape the benchmark times.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_1601_04633_amd import inputs


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a - b)


def _pair(oracle_mod, n, Ra, Pr, precision="fp64", seed=1601, amp=1e-4, **kw):
    from paper_1601_04633_amd.dmrt import Cavity
    okw = {k: v for k, v in kw.items()}
    bc = okw.pop("bc_mode", 0)
    o = oracle_mod.Oracle(n, Ra, Pr, bc=bc, **okw)
    c = Cavity(n=n, Ra=Ra, Pr=Pr, precision=precision, bc_mode=bc, **okw)
    th0 = inputs.theta_noise(n, seed, amp=amp)
    o.set_theta(th0)
    c.set_theta(th0)
    return o, c


def _compare_fields(o, c, tol, names=("U", "V", "theta", "P")):
    fo, fc = o.fields(), c.fields()
    errs = {nm: rel(b, a) for nm, a, b in zip(("U", "V", "theta", "P"), fo, fc)}
    bad = {k: v for k, v in errs.items() if k in names and not v <= tol}
    assert not bad, f"field errors {errs}"
    return errs


@pytest.mark.parametrize("n", [4, 5, 37, 64, 100, 130, 257])
def test_fp64_cavity_matches_oracle(oracle_mod, n):
    print(f"[parity] fp64 cavity n={n}", flush=True)
    o, c = _pair(oracle_mod, n, 1e4, 0.01)
    for steps in (1, 49, 150):
        o.step(steps)
        c.step(steps)
        _compare_fields(o, c, 1e-12)
    for wall in (0, 1):
        no, lo = o.nusselt(wall)
        nc, lc = c.nusselt(wall)
        assert abs(nc - no) <= 1e-12 * abs(no)
        assert rel(lc, lo) <= 1e-12


@pytest.mark.parametrize("bc,kw", [
    (1, dict(gbeta_override=1e-3, force_x=2e-6)),
    (2, dict(gbeta_override=0.0, force_x=1e-5)),
    (3, dict(theta_ref=0.2)),
    (0, dict(theta_ref=-0.5, a=0.3)),
    (0, dict(q5_mode=1, Ma=0.01)),
])
def test_fp64_wall_modes_match_oracle(oracle_mod, bc, kw):
    print(f"[parity] fp64 bc={bc} {kw}", flush=True)
    o, c = _pair(oracle_mod, 70, 1e4, 0.02, amp=0.05, bc_mode=bc, **kw)
    o.step(300)
    c.step(300)
    if bc == 2:
        # x-independent forced flow without buoyancy: V and P vanish in exact
        # arithmetic, so they are compared absolutely
        _compare_fields(o, c, 1e-12, names=("U", "theta"))
        for a, b in zip(o.fields()[1::2], c.fields()[1::2]):
            assert np.abs(a).max() < 1e-17 and np.abs(b).max() < 1e-17
    else:
        _compare_fields(o, c, 1e-12)


def test_fp64_hot_wall_profile_matches_oracle(oracle_mod):
    n = 48
    o, c = _pair(oracle_mod, n, 1e4, 0.01)
    tw = inputs.hot_wall_profile(n, 7)
    o.set_hot_wall(tw)
    c.set_hot_wall(tw)
    o.step(400)
    c.step(400)
    _compare_fields(o, c, 1e-12)
    assert rel(c.nusselt(0)[1], o.nusselt(0)[1]) <= 1e-12


def test_fp64_equilibrium_init_matches_oracle(oracle_mod):
    """Taylor-Green-like initial velocity through dmrt_set_equilibrium."""
    from paper_1601_04633_amd.dmrt import Cavity
    n = 40
    k = 2 * np.pi / n
    X, Y = np.meshgrid(np.arange(n), np.arange(n))
    U = -1e-3 * np.cos(k * X) * np.sin(k * Y)
    V = 1e-3 * np.sin(k * X) * np.cos(k * Y)
    T = 0.1 * np.sin(k * X)
    R = 1e-4 * np.cos(k * Y)
    o = oracle_mod.Oracle(n, 100.0, 1.0, bc=1, gbeta_override=1e-4)
    c = Cavity(n=n, Ra=100.0, Pr=1.0, bc_mode=1, gbeta_override=1e-4)
    o.set_equilibrium(drho=R, U=U, V=V, theta=T)
    c.set_equilibrium(drho=R, U=U, V=V, theta=T)
    _compare_fields(o, c, 1e-13)
    o.step(200)
    c.step(200)
    _compare_fields(o, c, 1e-12)


def test_config0_fp64_20000_steps(oracle_mod):
    """64^2, Ra 1e3, Pr 0.01, FP64, 20,000 steps from seeded noise: fields
    and hot-wall Nu within 1e-12 of the oracle."""
    print("[parity] config 64^2 fp64 20000 steps", flush=True)
    o, c = _pair(oracle_mod, 64, 1e3, 0.01)
    o.step(20000)
    c.step(20000)
    errs = _compare_fields(o, c, 1e-12)
    no, lo = o.nusselt(0)
    nc, lc = c.nusselt(0)
    assert abs(nc - no) <= 1e-12 * no, (nc, no, errs)


def _set_mode(c, mode):
    """The benchmark's launch shape (six steps per launch, workgroups of
    6 x 2 wavefronts marching up chunks of rows), the four-step marching
    form (4 x 3 wavefronts) or the tile form (64 x 16 footprints);
    die-aware order and graphs of 60 steps in all."""
    c.set_launch(256, 1, 1, 60)
    if mode == "march6":
        c.set_temporal_march(6, 2, 0)
    elif mode == "march":
        c.set_temporal_march(4, 3, 0)
    else:
        c.set_temporal(4, 16)


@pytest.fixture(scope="module")
def oracle_1024(oracle_mod):
    """The oracle's fields of the 1024^2, Ra 1e5, Pr 0.001 cavity after 52
    steps from the seeded noise (1M nodes per step: ~6 s on one core)."""
    print("[parity] oracle 1024^2, 52 steps", flush=True)
    o = oracle_mod.Oracle(1024, 1e5, 0.001)
    o.set_theta(inputs.theta_noise(1024, 1601))
    o.step(52)
    return o.fields(), o.nusselt(0)[0]


@pytest.mark.parametrize("mode", ["march6", "march", "tile"])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_full_size_1024_matches_oracle(oracle_1024, precision, tol, mode):
    """1024^2, Ra 1e5, Pr 0.001 in the benchmark's launch shape (and the
    four-step marching and tile forms): U, V, theta, P and the hot-wall Nu
    after 52 steps (eight six-step launches and a remainder, or 13
    four-step launches; a graph of 60 steps not yet reached) within the
    precision's bar of the oracle."""
    from paper_1601_04633_amd.dmrt import Cavity
    print(f"[parity] 1024^2 {precision} {mode}", flush=True)
    c = Cavity(n=1024, Ra=1e5, Pr=0.001, precision=precision)
    _set_mode(c, mode)
    c.set_theta(inputs.theta_noise(1024, 1601))
    c.step(52)
    fo, nu_o = oracle_1024
    fc = c.fields()
    nu_c = c.nusselt(0)[0]
    c.close()
    errs = {nm: rel(b, a) for nm, a, b in zip(("U", "V", "theta", "P"), fo, fc)}
    print(f"[parity] 1024^2 {precision} {mode}: " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items())
          + f", Nu {abs(nu_c / nu_o - 1):.2e}", flush=True)
    assert all(v <= tol for v in errs.values()), errs
    assert abs(nu_c - nu_o) <= (1e-12 if precision == "fp64" else 1e-4) * abs(nu_o)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("n,temporal", [(1024, ("march", 4, 3, 0)), (1024, ("tile", 4, 16)),
                                        (1024, ("march", 6, 2, 0)), (2048, ("march", 6, 2, 0))])
def test_full_size_multi_step_equals_single_steps(precision, n, temporal):
    """The launch shapes at full size (six steps per launch on marching
    workgroups with the automatic chunk — the benchmark's —, four steps per
    launch marching and in tiles), 4,000 steps (1,200 at 2048^2) from theta noise of
    amplitude 1e-2: bitwise the state of one step per launch."""
    from paper_1601_04633_amd.dmrt import Cavity
    steps = 4000 if n == 1024 else 1200
    print(f"[parity] {n}^2 {precision} {temporal} vs single steps, {steps} steps", flush=True)
    th0 = inputs.theta_noise(n, 4000 + n, amp=1e-2)
    out = []
    for mode in (None, temporal):
        c = Cavity(n=n, Ra=1e5, Pr=0.001, precision=precision)
        c.set_launch(256, 1, 1, 60)
        if mode and mode[0] == "march":
            c.set_temporal_march(*mode[1:])
        elif mode:
            c.set_temporal(*mode[1:])
        c.set_theta(th0)
        c.step(steps)
        out.append(c.raw_state())
        c.close()
    (fa, ga), (fb, gb) = out
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)
    assert np.isfinite(fa).all() and np.abs(fa).max() > 0


def test_fp32_vs_fp64_steady_config0():
    """FP32 storage as deviations from w_i rho0 vs FP64 on the GPU, steady
    64^2 case after 20,000 steps: <= 1e-5 on U, V, theta, <= 1e-4 on Nu."""
    from paper_1601_04633_amd.dmrt import Cavity
    th0 = inputs.theta_noise(64, 1601)
    res = {}
    for prec in ("fp32", "fp64"):
        c = Cavity(n=64, Ra=1e3, Pr=0.01, precision=prec)
        c.set_theta(th0)
        c.step(20000)
        res[prec] = (c.fields(), c.nusselt(0)[0])
    (f32, n32), (f64, n64) = res["fp32"], res["fp64"]
    for nm, a, b in zip(("U", "V", "theta"), f32[:3], f64[:3]):
        assert rel(a, b) <= 1e-5, (nm, rel(a, b))
    assert abs(n32 - n64) <= 1e-4 * n64


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_launch_shape_does_not_change_results(precision):
    """Block shape, die-aware tile order and graph capture change only the
    schedule: results are bitwise identical."""
    from paper_1601_04633_amd.dmrt import Cavity
    n = 200
    th0 = inputs.theta_noise(n, 3, amp=1e-2)
    ref = None
    for shape in [(256, 1, 1, 64), (64, 4, 0, 0), (128, 2, 1, 10), (512, 2, 0, 64), (64, 1, 1, 0)]:
        c = Cavity(n=n, Ra=1e4, Pr=0.005, precision=precision)
        c.set_launch(*shape)
        c.set_theta(th0)
        c.step(333)
        f, g = c.raw_state()
        if ref is None:
            ref = (f, g)
        else:
            assert np.array_equal(f, ref[0]) and np.array_equal(g, ref[1]), shape


def test_checkpoint_resume_is_bitwise():
    from paper_1601_04633_amd.dmrt import Cavity
    n = 96
    th0 = inputs.theta_noise(n, 11)
    a = Cavity(n=n, Ra=1e4, Pr=0.01, precision="fp32")
    a.set_theta(th0)
    a.step(101)
    blob = a.save_state()
    a.step(250)
    b = Cavity(n=n, Ra=1e4, Pr=0.01, precision="fp32")
    b.load_state(blob)
    assert b.steps == 101
    b.step(250)
    fa, ga = a.raw_state()
    fb, gb = b.raw_state()
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)


def test_nu_series_matches_direct_calls():
    from paper_1601_04633_amd.dmrt import Cavity
    n = 64
    th0 = inputs.theta_noise(n, 12)
    a = Cavity(n=n, Ra=1e4, Pr=0.01)
    a.set_theta(th0)
    a.nu_series(7, 1000)
    a.set_launch(256, 1, 1, 28)
    a.step(7 * 40 + 3)
    series = a.nu_series_read()
    assert len(series) == 40
    b = Cavity(n=n, Ra=1e4, Pr=0.01)
    b.set_theta(th0)
    direct = []
    for _ in range(40):
        b.step(7)
        direct.append(b.nusselt(0)[0])
    np.testing.assert_array_equal(series, np.array(direct))


def test_residual_and_watchdog():
    from paper_1601_04633_amd.dmrt import Cavity
    n = 32
    c = Cavity(n=n, Ra=1e4, Pr=0.01, precision="fp32")
    c.set_theta(inputs.theta_noise(n, 13))
    c.residual()
    c.step(10)
    rt, ru, bad = c.residual()
    assert rt > 0 and ru > 0 and not bad
    rt2, ru2, bad = c.residual()
    assert rt2 == 0.0 and ru2 == 0.0 and not bad
    # plant a NaN in a checkpoint blob: the watchdog reports it
    blob = bytearray(c.save_state())
    off = 8 * 8 + n * 8 + 4 * 17
    blob[off:off + 4] = np.array([np.nan], dtype=np.float32).tobytes()
    c.load_state(bytes(blob))
    _, _, bad = c.residual()
    assert bad


WATCHDOG_FORMS = {"single": (1, 10), "tile": (4, 12), "march6": ("march", 6, 2, 0)}


def _set_form(c, form):
    t = WATCHDOG_FORMS[form]
    if t[0] == "march":
        c.set_temporal_march(*t[1:])
    else:
        c.set_temporal(*t)


@pytest.mark.parametrize("form", list(WATCHDOG_FORMS))
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_step_watchdog_reports_nonfinite_state(precision, form):
    """dmrt_step's watchdog (the two isothermal-wall columns of the state a
    call starts from, checked by its first launch; dmrt_sync checks the
    current state) reports a NaN planted in the interior once it has spread
    to a wall: dmrt_sync returns DMRT_ENONFINITE, later dmrt_step calls
    return it without enqueuing, and re-initialising clears it; a healthy
    run never reports it."""
    from paper_1601_04633_amd.dmrt import Cavity, DmrtError, DMRT_ENONFINITE
    n = 40
    c = Cavity(n=n, Ra=1e4, Pr=0.01, precision=precision)
    _set_form(c, form)
    c.set_theta(inputs.theta_noise(n, 16))
    c.step(300)
    c.sync()
    esz = 8 if precision == "fp64" else 4
    blob = bytearray(c.save_state())
    # g plane 2 (index 9 + 2 of the 14), node (x, y) = (20, 17): interior
    off = 8 * 8 + n * 8 + esz * ((9 + 2) * n * n + 17 * n + 20)
    blob[off:off + esz] = np.array([np.nan], dtype=np.float64 if esz == 8 else np.float32).tobytes()
    c.load_state(bytes(blob))
    c.step(2)                          # the NaN has not reached a wall column yet
    c.sync()
    c.step(2 * n)
    with pytest.raises(DmrtError) as e:
        c.sync()
    assert e.value.code == DMRT_ENONFINITE
    with pytest.raises(DmrtError) as e:
        c.step(10)
    assert e.value.code == DMRT_ENONFINITE
    c.set_theta(inputs.theta_noise(n, 16))
    c.step(100)
    c.sync()
    c.close()


def test_step_counts_not_multiple_of_k_full_size():
    """The benchmark's cavity (1024^2 FP32, six steps per launch): counts
    20, 13 and 7 (launches of 6+6+4+4, 6+4+3 and 4+3 steps) give bitwise the
    state of single steps."""
    from paper_1601_04633_amd.dmrt import Cavity
    n = 1024
    th0 = inputs.theta_noise(n, 1601, amp=1e-2)
    counts = [20, 13, 7]
    print(f"[parity] 1024^2 step counts {counts} in six-step marching vs single steps", flush=True)
    out = []
    for march in (False, True):
        c = Cavity(n=n, Ra=1e5, Pr=0.001, precision="fp32")
        if march:
            c.set_temporal_march(6, 2, 0)
        c.set_launch(256, 1, 1, 0)
        c.set_theta(th0)
        for k in counts:
            c.step(k)
        out.append(c.raw_state())
        c.close()
    (fa, ga), (fb, gb) = out
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)


@pytest.mark.parametrize("form,n", [(f, 40) for f in WATCHDOG_FORMS] + [("march6", 1024)])
def test_step_watchdog_in_first_launch(form, n):
    """Without dmrt_sync: the check that the first launch of a dmrt_step
    call runs on the state it starts from sets the flag, and the next call
    returns DMRT_ENONFINITE (graphs off, so every call starts with a
    stepping launch).  A NaN placed on a wall column is found by the first
    call after it (at 1024^2 in the last of the three workgroups that the
    six-step launch appends)."""
    import torch
    from paper_1601_04633_amd.dmrt import Cavity, DmrtError, DMRT_ENONFINITE
    c = Cavity(n=n, Ra=1e4, Pr=0.01, precision="fp32")
    _set_form(c, form)
    c.set_launch(256, 1, 1, 0)
    c.set_theta(inputs.theta_noise(n, 16))
    c.step(30)
    c.sync()
    blob = bytearray(c.save_state())
    # f plane 3 at node (x, y) = (n - 1, yw): on the cold wall, in the
    # last rows (wall node 2 yw + 1 of the check's 2n)
    yw = n - 15
    off = 8 * 8 + n * 8 + 4 * (3 * n * n + yw * n + n - 1)
    blob[off:off + 4] = np.array([np.inf], dtype=np.float32).tobytes()
    c.load_state(bytes(blob))
    c.step(7)                          # its first launch finds the wall value
    torch.cuda.synchronize()           # the flag is written; no dmrt_sync
    with pytest.raises(DmrtError) as e:
        c.step(1)
    assert e.value.code == DMRT_ENONFINITE
    c.close()


def _host_residual(prev, now):
    """||theta_now - theta_prev|| / ||theta_now|| and the same for (U, V),
    from (U, V, theta) snapshots."""
    (u0, v0, t0), (u1, v1, t1) = prev, now
    rt = np.sqrt(((t1 - t0) ** 2).sum() / (t1 ** 2).sum())
    ru = np.sqrt((((u1 - u0) ** 2).sum() + ((v1 - v0) ** 2).sum()) / ((u1 ** 2).sum() + (v1 ** 2).sum()))
    return rt, ru


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_residual_value_matches_host_norms(oracle_mod, precision):
    """dmrt_residual (the convergence measure used to decide steady state)
    equals ||x_now - x_prev||_2 / ||x_now||_2 for theta and for (U, V),
    computed on the host from two dmrt_get_fields snapshots, to 1e-12; in
    FP64 also from the oracle's fields at the same steps."""
    from paper_1601_04633_amd.dmrt import Cavity
    n = 57
    th0 = inputs.theta_noise(n, 15, amp=1e-2)
    c = Cavity(n=n, Ra=1e4, Pr=0.01, precision=precision)
    c.set_theta(th0)
    o = oracle_mod.Oracle(n, 1e4, 0.01)
    o.set_theta(th0)
    c.step(5)
    o.step(5)
    # the first call compares against zero: exactly 1
    rt, ru, bad = c.residual()
    assert rt == 1.0 and ru == 1.0 and not bad
    snaps = [c.fields()[:3]]
    osnaps = [o.fields()[:3]]
    for k in (1, 37, 400):
        c.step(k)
        o.step(k)
        rt, ru, bad = c.residual()
        snaps.append(c.fields()[:3])
        osnaps.append(o.fields()[:3])
        et, eu = _host_residual(snaps[-2], snaps[-1])
        print(f"[parity] residual {precision} after +{k}: theta {rt:.6e} (host {et:.6e}), "
              f"u {ru:.6e} (host {eu:.6e})", flush=True)
        assert not bad
        assert abs(rt - et) <= 1e-12 * et and abs(ru - eu) <= 1e-12 * eu
        if precision == "fp64":
            ot, ou = _host_residual(osnaps[-2], osnaps[-1])
            assert abs(rt - ot) <= 1e-10 * ot and abs(ru - ou) <= 1e-10 * ou
    c.close()


def test_torch_buffers_and_stream(oracle_mod):
    import torch
    from paper_1601_04633_amd.dmrt import Cavity
    n = 80
    th0 = inputs.theta_noise(n, 14)
    a = Cavity(n=n, Ra=1e4, Pr=0.01, torch_buffers=True)
    a.set_theta(th0)
    a.step(120)
    b = Cavity(n=n, Ra=1e4, Pr=0.01)
    b.set_theta(th0)
    b.step(120)
    fa, ga = a.raw_state()
    fb, gb = b.raw_state()
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)
    f_ptr, _, _ = a.buffers()
    assert f_ptr == a._tensors[0].data_ptr()


def test_case1_physics_against_paper():
    """The paper's Case 1 (Ra 1e4, Pr 0.01): steady Nu_avg 1.95, Nu_max 3.02
    at Y = 0.30 (Section 4).  FP64 at 128^2 to Fo = 4."""
    import json, os
    from paper_1601_04633_amd.dmrt import Cavity
    case = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                       "paper_values.json")))["cases"][0]
    n = 128
    c = Cavity(n=n, Ra=case["Ra"], Pr=case["Pr"])
    c.set_theta(inputs.theta_noise(n, 1601))
    steps = int(4 * n * n / c.derived()["alpha"])
    c.step(steps)
    nu, loc = c.nusselt(0)
    nuc, _ = c.nusselt(1)
    y = (np.arange(n) + 0.5) / n
    print(f"[physics] case 1 n={n}: Nu {nu:.5f} cold {nuc:.5f} max {loc.max():.4f} at {y[loc.argmax()]:.4f}")
    assert abs(nu / case["nu_avg"] - 1) < 0.01
    assert abs(loc.max() / case["nu_max"] - 1) < 0.01
    assert abs(y[loc.argmax()] - case["y_nu_max"]) < 0.02
    assert abs(nuc / nu - 1) < 1e-6


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("k,rows", [(2, 4), (2, 6), (2, 10), (2, 16), (3, 6), (3, 10), (3, 12),
                                    (3, 14), (3, 16), (4, 10), (4, 12), (4, 14), (4, 16)])
def test_multi_step_launch_equals_single_steps(precision, k, rows):
    """K steps per launch through LDS give bitwise the state of single
    steps, for ragged sizes, odd step counts, graph replay and Nu sampling
    that splits groups."""
    from paper_1601_04633_amd.dmrt import Cavity
    for n in (4, 5, 37, 62, 63, 100, 130, 257):
        th0 = inputs.theta_noise(n, 40 + n, amp=1e-2)
        ref = Cavity(n=n, Ra=2e4, Pr=0.01, precision=precision)
        ref.set_theta(th0)
        ref.nu_series(7, 100)
        ref.step(131)
        two = Cavity(n=n, Ra=2e4, Pr=0.01, precision=precision)
        two.set_temporal(k, rows)
        two.set_theta(th0)
        two.nu_series(7, 100)
        two.step(67)
        two.step(64)
        fa, ga = ref.raw_state()
        fb, gb = two.raw_state()
        assert np.array_equal(fa, fb) and np.array_equal(ga, gb), (n, k, rows)
        np.testing.assert_array_equal(ref.nu_series_read(), two.nu_series_read())


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("k,group", [(2, 8), (3, 2), (3, 4), (4, 1), (4, 2), (4, 3), (4, 4), (6, 2)])
def test_marching_launch_equals_single_steps(precision, k, group):
    """K steps per launch with workgroups marching up chunks of rows give
    bitwise the state of single steps: ragged sizes, chunks of one row, of a
    few rows, not dividing n, the whole height and the automatic choice,
    odd step counts, graph replay and Nu sampling that splits groups.  A
    pair whose LDS rings exceed a workgroup's 160 KB in this precision is
    rejected."""
    from paper_1601_04633_amd.dmrt import Cavity, DmrtError
    esz = 8 if precision == "fp64" else 4
    if (k - 1) * 14 * (group + 2) * 64 * esz > 160 * 1024:
        c = Cavity(n=32, Ra=2e4, Pr=0.01, precision=precision)
        with pytest.raises(DmrtError):
            c.set_temporal_march(k, group, 0)
        c.close()
        return
    for n, chunk in ((4, 0), (5, 1), (37, 5), (63, 0), (100, 7), (130, 37), (257, 0), (70, 70)):
        print(f"[parity] march K={k} B={group} n={n} chunk={chunk} {precision}", flush=True)
        th0 = inputs.theta_noise(n, 40 + n, amp=1e-2)
        ref = Cavity(n=n, Ra=2e4, Pr=0.01, precision=precision)
        ref.set_theta(th0)
        ref.nu_series(7, 100)
        ref.step(131)
        m = Cavity(n=n, Ra=2e4, Pr=0.01, precision=precision)
        used = m.set_temporal_march(k, group, chunk)
        assert (chunk == 0 and 1 <= used <= n) or used == min(chunk, n)
        assert m.temporal_march() == (group, used)
        m.set_theta(th0)
        m.nu_series(7, 100)
        m.step(67)
        m.step(64)
        fa, ga = ref.raw_state()
        fb, gb = m.raw_state()
        assert np.array_equal(fa, fb) and np.array_equal(ga, gb), (n, k, group, chunk)
        np.testing.assert_array_equal(ref.nu_series_read(), m.nu_series_read())
        ref.close()
        m.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("temporal", [(4, 16), (3, 12), ("march", 4, 3, 0), ("march", 6, 2, 0),
                                      ("march", 4, 1, 9)])
def test_nu_series_inside_multi_step_launches(precision, temporal):
    """A Nusselt sample due on any step of a K-step launch is taken by that
    launch (wall-column sums of the step into a slot; the slots of many
    launches reduced into the ring by one kernel, in step order): the
    series equals that of single steps bitwise, for strides shorter than,
    equal to, coprime with and longer than K, with and without graph
    replay, and the state is unchanged by the sampling."""
    from paper_1601_04633_amd.dmrt import Cavity
    n, steps = 100, 257
    th0 = inputs.theta_noise(n, 77, amp=1e-2)
    # (stride, graph steps): samples of many launches are reduced together,
    # in slots that run out mid-range for stride 1
    for stride, graph in ((1, 60), (1, 0), (2, 60), (3, 60), (7, 60), (7, 0), (10, 60)):
        print(f"[parity] nu series inside {temporal} stride {stride} graph {graph} {precision}", flush=True)
        out = []
        for mode in (None, temporal):
            c = Cavity(n=n, Ra=2e4, Pr=0.01, precision=precision)
            if mode and mode[0] == "march":
                c.set_temporal_march(*mode[1:])
            elif mode:
                c.set_temporal(*mode)
            c.set_launch(256, 1, 1, graph)
            c.set_theta(th0)
            c.nu_series(stride, 400)
            c.step(steps)
            out.append((c.nu_series_read(), c.raw_state()))
            c.close()
        (sa, (fa, ga)), (sb, (fb, gb)) = out
        assert len(sa) == steps // stride
        np.testing.assert_array_equal(sa, sb)
        assert np.array_equal(fa, fb) and np.array_equal(ga, gb)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("temporal", [("march", 6, 2, 0), ("march", 4, 3, 0), ("march", 4, 2, 11)])
def test_step_counts_not_multiple_of_k(precision, temporal):
    """Counts that are not a multiple of K end in marching launches of fewer
    steps (e.g. 20 = 6 + 6 + 4 + 4 for K = 6): every count from 1 to 13, then
    17 and 20, called one after another, gives bitwise the state and the
    Nusselt series (a sample every 3 steps) of single steps, without graphs
    so that each call plans its own launches."""
    from paper_1601_04633_amd.dmrt import Cavity
    n = 100
    th0 = inputs.theta_noise(n, 91, amp=1e-2)
    counts = list(range(1, 14)) + [17, 20]
    print(f"[parity] step counts {counts} in {temporal} {precision}", flush=True)
    out = []
    for mode in (None, temporal):
        c = Cavity(n=n, Ra=2e4, Pr=0.01, precision=precision)
        if mode:
            c.set_temporal_march(*mode[1:])
        c.set_launch(256, 1, 1, 0)
        c.set_theta(th0)
        c.nu_series(3, 100)
        for k in counts:
            c.step(k)
        out.append((c.nu_series_read(), c.raw_state()))
        c.close()
    (sa, (fa, ga)), (sb, (fb, gb)) = out
    assert len(sa) == sum(counts) // 3
    np.testing.assert_array_equal(sa, sb)
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)


def test_marching_fp64_matches_oracle(oracle_mod):
    o, c = _pair(oracle_mod, 100, 1e4, 0.01)
    c.set_temporal_march(4, 4, 0)
    o.step(151)
    c.step(151)
    _compare_fields(o, c, 1e-12)


@pytest.mark.parametrize("k,rows", [(2, 10), (3, 10), (4, 16)])
def test_multi_step_fp64_matches_oracle(oracle_mod, k, rows):
    o, c = _pair(oracle_mod, 100, 1e4, 0.01)
    c.set_temporal(k, rows)
    o.step(151)
    c.step(151)
    _compare_fields(o, c, 1e-12)


def test_two_step_rejected_outside_cavity():
    from paper_1601_04633_amd.dmrt import Cavity, DmrtError
    c = Cavity(n=32, Ra=1e4, Pr=0.01, bc_mode=1)
    with pytest.raises(DmrtError):
        c.set_temporal(2, 10)


def test_marching_rejects_bad_arguments():
    from paper_1601_04633_amd.dmrt import Cavity, DmrtError
    c = Cavity(n=32, Ra=1e4, Pr=0.01)
    for args in ((4, 5, 0), (1, 4, 0), (5, 2, 0), (8, 2, 0), (4, 4, -1), (2, 4, 0)):
        with pytest.raises(DmrtError):
            c.set_temporal_march(*args)
    assert c.temporal_march() == (0, 0)
    c.set_temporal_march(4, 4, 10)
    c.set_temporal(4, 16)                      # tile kernel again: marching off
    assert c.temporal_march() == (0, 0)
    c.close()
    p = Cavity(n=32, Ra=1e4, Pr=0.01, bc_mode=1)
    with pytest.raises(DmrtError):
        p.set_temporal_march(4, 4, 0)
    p.close()


@pytest.mark.parametrize("mode", ["march6", "march", "tile"])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_full_size_centro_symmetry_in_benchmark_shape(precision, mode):
    """1024^2, Ra 1e5, Pr 0.001 in the benchmark's launch shape (and the
    four-step marching and tile forms), 4,000 steps from theta = 0:
    rotating the cavity by 180 degrees and flipping theta maps the problem
    onto itself, so theta, U, V
    stay antisymmetric and P symmetric at full size (a property that holds
    at any size, where the oracle cannot follow)."""
    from paper_1601_04633_amd.dmrt import Cavity
    print(f"[parity] 1024^2 centro-symmetry {precision} {mode}", flush=True)
    n = 1024
    c = Cavity(n=n, Ra=1e5, Pr=0.001, precision=precision)
    _set_mode(c, mode)
    c.set_theta(np.zeros((n, n)))
    c.step(4000)
    U, V, T, P = c.fields()
    c.close()
    R = lambda A: A[::-1, ::-1]
    tol = 1e-6 if precision == "fp32" else 1e-13
    assert np.abs(T + R(T)).max() <= tol * np.abs(T).max()
    assert np.abs(U + R(U)).max() <= tol * np.abs(U).max()
    assert np.abs(V + R(V)).max() <= tol * np.abs(V).max()
    assert np.abs(P - R(P)).max() <= tol * np.abs(P).max()
    # the boundary layers have formed: rising at the hot wall, sinking at the cold
    assert V[n // 2, 0] > 0 and V[n // 2, n - 1] < 0 and np.abs(U).max() > 1e-5
