"""GPU tests of the hand-written adjoint (gradient of the time-averaged
hot-wall Nusselt number with respect to the hot-wall profile and the initial
temperature field):

* one step, and a few hundred steps with several checkpoint segments, against
  the CPU reference gradient (automatic differentiation of a vectorised FP64
  restatement of the oracle; oracle/torch_ref.py);
* the 32^2, 10,000-step instance against FP64 central differences of the C
  oracle (h = 1e-6): all 32 hot-wall entries, 64 initial-field entries and 4
  random directions;
* independence of the checkpoint interval (bitwise), the FP32 path at the
  256^2 configuration against the FP64 one, and the autograd Function.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_1601_04633_amd import inputs


def _cavity(n, Ra, Pr, precision="fp64", **kw):
    from paper_1601_04633_amd.dmrt import Cavity
    return Cavity(n=n, Ra=Ra, Pr=Pr, precision=precision, **kw)


def _gpu_grad(n, Ra, Pr, tw, t0, N, K, C, precision="fp64"):
    c = _cavity(n, Ra, Pr, precision)
    c.set_hot_wall(tw)
    c.set_theta(t0)
    J, gw, g0 = c.adjoint_nu(N, K, C)
    c.close()
    return J, gw, g0


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


@pytest.mark.parametrize("n", [16, 37])
def test_single_step_against_reference(n):
    from oracle.torch_ref import Reference
    print(f"[adjoint] single step n={n}", flush=True)
    tw = inputs.hot_wall_profile(n, 21)
    t0 = inputs.theta_noise(n, 22, amp=0.05)
    Jg, gw, g0 = _gpu_grad(n, 1e4, 0.01, tw, t0, 1, 1, 1)
    Jr, rw, r0 = Reference(n, 1e4, 0.01).gradient(tw, t0, 1, 1)
    assert abs(Jg - Jr) <= 1e-13 * abs(Jr)
    assert rel(gw, rw) <= 1e-12 and rel(g0, r0) <= 1e-12


@pytest.mark.parametrize("n,N,K,C", [(32, 600, 150, 100), (40, 333, 333, 64)])
def test_many_steps_against_reference(n, N, K, C):
    from oracle.torch_ref import Reference
    print(f"[adjoint] n={n} N={N} K={K} C={C}", flush=True)
    tw = inputs.hot_wall_profile(n, 23)
    t0 = inputs.theta_noise(n, 24, amp=1e-2)
    Jg, gw, g0 = _gpu_grad(n, 1e4, 0.01, tw, t0, N, K, C)
    Jr, rw, r0 = Reference(n, 1e4, 0.01).gradient(tw, t0, N, K, segment=100)
    assert abs(Jg - Jr) <= 1e-12 * abs(Jr)
    assert rel(gw, rw) <= 1e-10, rel(gw, rw)
    assert rel(g0, r0) <= 1e-10, rel(g0, r0)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_checkpoint_interval_does_not_change_gradients(precision):
    """The recompute reproduces the forward bitwise, so the gradients do not
    depend on the checkpoint interval (C = 1 recomputes nothing)."""
    n, N, K = 24, 300, 100
    tw = inputs.hot_wall_profile(n, 25)
    t0 = inputs.theta_noise(n, 26, amp=1e-2)
    ref = None
    for C in (1, 7, 50, 300):
        out = _gpu_grad(n, 1e4, 0.01, tw, t0, N, K, C, precision)
        if ref is None:
            ref = out
        else:
            assert out[0] == ref[0]
            assert np.array_equal(out[1], ref[1]) and np.array_equal(out[2], ref[2]), C


def test_fp64_adjoint_against_oracle_finite_differences(oracle_mod):
    """The 32^2 instance (Ra 1e4, Pr 0.01, FP64, 10,000 steps, mean Nu over
    the last 2,000, checkpoints every 500): adjoint gradients against
    central differences (h = 1e-6) of the C oracle's objective."""
    from oracle import fd
    n, Ra, Pr, N, K, C = 32, 1e4, 0.01, 10000, 2000, 500
    tw = inputs.hot_wall_profile(n, 1601)
    t0 = inputs.theta_noise(n, 1601)
    print("[adjoint] fd check 32^2 10000 steps", flush=True)
    Jg, gw, g0 = _gpu_grad(n, Ra, Pr, tw, t0, N, K, C)
    o = oracle_mod.Oracle(n, Ra, Pr)
    o.set_hot_wall(tw)
    o.set_theta(t0)
    Jo = o.objective(N, K)
    assert abs(Jg - Jo) <= 1e-12 * abs(Jo)
    rng = np.random.default_rng(1601)
    # (a) every hot-wall entry and 4 random directions, h = 1e-6
    dirs, adj = [], []
    for y in range(n):
        dirs.append((np.eye(n)[y], np.zeros((n, n))))
        adj.append(gw[y])
    dw_all = inputs.random_directions((n,), 4, 77)
    d0_all = inputs.random_directions((n, n), 4, 78)
    for dw, d0 in zip(dw_all, d0_all):
        dirs.append((dw / np.sqrt(2), d0 / np.sqrt(2)))
        adj.append(((gw * dw).sum() + (g0 * d0).sum()) / np.sqrt(2))
    got = np.array(fd.directional_derivatives(n, Ra, Pr, tw, t0, N, K, dirs, h=1e-6, workers=16))
    adj = np.array(adj)
    rel_a = np.abs(adj - got) / np.abs(got)
    print(f"[adjoint] fd (theta_w, directions; h 1e-6): max rel err {rel_a.max():.3e}", flush=True)
    assert rel_a.max() <= 1e-6, rel_a.max()
    # (b) the initial field.  After 10,000 steps these derivatives are
    # 1e-9..2e-5, below the round-off of a central difference at h = 1e-6;
    # J is linear in theta0 to ~1e-9 at h = 1e-2, where the round-off floor
    # of a difference is ~2e-13 absolute.  Dense random directions (whose
    # derivatives are far above that floor) must agree to 1e-6 relative,
    # and 64 single entries as a vector (normwise) to 1e-6.
    dirs = [(np.zeros(n), d0) for d0 in inputs.random_directions((n, n), 4, 79)]
    adj = np.array([(g0 * d0).sum() for _, d0 in dirs])
    got = np.array(fd.directional_derivatives(n, Ra, Pr, tw, t0, N, K, dirs, h=1e-2, workers=16))
    rel_d = np.abs(adj - got) / np.abs(got)
    print(f"[adjoint] fd (theta0 directions; h 1e-2): |d| {np.abs(got).min():.2e}..{np.abs(got).max():.2e}, "
          f"max rel err {rel_d.max():.3e}", flush=True)
    assert rel_d.max() <= 1e-6, rel_d
    dirs, adj = [], []
    for idx in rng.choice(n * n, size=64, replace=False):
        d0 = np.zeros(n * n)
        d0[idx] = 1.0
        dirs.append((np.zeros(n), d0.reshape(n, n)))
        adj.append(g0.reshape(-1)[idx])
    got = np.array(fd.directional_derivatives(n, Ra, Pr, tw, t0, N, K, dirs, h=1e-2, workers=16))
    adj = np.array(adj)
    err = np.abs(adj - got)
    print(f"[adjoint] fd (theta0 entries; h 1e-2): normwise rel err "
          f"{np.linalg.norm(err) / np.linalg.norm(got):.3e}, max abs err {err.max():.3e}, "
          f"|grad| {np.abs(got).min():.2e}..{np.abs(got).max():.2e}", flush=True)
    assert np.linalg.norm(err) <= 1e-6 * np.linalg.norm(got)


def test_fp64_adjoint_config_instance_against_reference():
    """The same 32^2, 10,000-step instance against the CPU FP64 reference
    adjoint (tests/golden/adjoint_ref_32.json, written from
    oracle/torch_ref.py alone): J to 1e-12, both gradients to 1e-10
    relative (normwise), with one checkpoint every 500 steps and four
    adjoint steps per backward launch."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "adjoint_ref_32.json")))
    n, Ra, Pr, N, K = gold["n"], gold["Ra"], gold["Pr"], gold["steps"], gold["avg_last"]
    tw = inputs.hot_wall_profile(n, gold["hot_wall_seed"])
    t0 = inputs.theta_noise(n, gold["theta0_seed"])
    rw = np.array(gold["dJ_dthetaw"])
    r0 = np.array(gold["dJ_dtheta0"]).reshape(n, n)
    for temporal in ((1, 10), (4, 12)):
        c = _cavity(n, Ra, Pr)
        c.adjoint_set_temporal(*temporal)
        c.set_hot_wall(tw)
        c.set_theta(t0)
        Jg, gw, g0 = c.adjoint_nu(N, K, 500)
        c.close()
        print(f"[adjoint] 32^2 x 10000 vs reference, backward {temporal}: J {abs(Jg / gold['J'] - 1):.2e}, "
              f"dJ/dtheta_w {rel(gw, rw):.2e}, dJ/dtheta0 {rel(g0, r0):.2e}", flush=True)
        assert abs(Jg - gold["J"]) <= 1e-12 * abs(gold["J"])
        assert rel(gw, rw) <= 1e-10 and rel(g0, r0) <= 1e-10


def test_fp32_adjoint_config_against_fp64():
    """256^2, Ra 1e4, Pr 0.01, 10,000 steps, mean Nu over the last 2,000,
    checkpoints every 500: the FP32 path against the FP64 path."""
    n, Ra, Pr, N, K, C = 256, 1e4, 0.01, 10000, 2000, 500
    tw = inputs.hot_wall_profile(n, 4633)
    t0 = inputs.theta_noise(n, 1601)
    print("[adjoint] fp32 vs fp64 256^2", flush=True)
    J32, w32, z32 = _gpu_grad(n, Ra, Pr, tw, t0, N, K, C, "fp32")
    J64, w64, z64 = _gpu_grad(n, Ra, Pr, tw, t0, N, K, C, "fp64")
    print(f"[adjoint] fp32 vs fp64: J {abs(J32 - J64) / abs(J64):.2e}, dJ/dtheta_w "
          f"{rel(w32, w64):.2e}, dJ/dtheta0 {rel(z32, z64):.2e}", flush=True)
    # measured: 1.1e-5, 6.5e-6, 1.1e-7; bars about ten times those
    assert abs(J32 - J64) <= 1e-4 * abs(J64)
    assert rel(w32, w64) <= 1e-4
    assert rel(z32, z64) <= 1e-6


def test_autograd_function():
    import torch
    from paper_1601_04633_amd.adjoint import nu_objective
    n, N, K, C = 32, 400, 100, 50
    tw = torch.tensor(inputs.hot_wall_profile(n, 27), requires_grad=True)
    t0 = torch.tensor(inputs.theta_noise(n, 28, amp=1e-2), requires_grad=True)
    c = _cavity(n, 1e4, 0.01)
    J = nu_objective(tw, t0, c, N, K, C)
    (2.0 * J).backward()
    Jd, gw, g0 = _gpu_grad(n, 1e4, 0.01, tw.detach().numpy(), t0.detach().numpy(), N, K, C)
    assert float(J.detach()) == Jd
    assert np.array_equal(tw.grad.numpy(), 2.0 * gw)
    assert np.array_equal(t0.grad.numpy(), 2.0 * g0)
    c.close()


def test_autograd_function_float32_and_device_inputs():
    """FP32 leaf tensors on the GPU get FP32 gradients on the GPU (the
    values of the FP64 adjoint rounded once)."""
    import torch
    from paper_1601_04633_amd.adjoint import nu_objective
    n, N, K, C = 16, 60, 20, 20
    tw64 = inputs.hot_wall_profile(n, 31)
    t064 = inputs.theta_noise(n, 32, amp=1e-2)
    tw = torch.tensor(tw64, dtype=torch.float32, device="cuda", requires_grad=True)
    t0 = torch.tensor(t064, dtype=torch.float32, device="cuda", requires_grad=True)
    c = _cavity(n, 1e4, 0.01)
    J = nu_objective(tw, t0, c, N, K, C)
    J.backward()
    c.close()
    assert tw.grad.dtype == torch.float32 and tw.grad.device.type == "cuda"
    assert t0.grad.dtype == torch.float32 and t0.grad.device.type == "cuda"
    _, gw, g0 = _gpu_grad(n, 1e4, 0.01, tw.detach().cpu().double().numpy(),
                          t0.detach().cpu().double().numpy(), N, K, C)
    assert np.array_equal(tw.grad.cpu().numpy(), gw.astype(np.float32))
    assert np.array_equal(t0.grad.cpu().numpy(), g0.astype(np.float32))


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_multi_step_forward_does_not_change_gradients(precision):
    """The checkpointed forward may take K steps per launch (tile or
    row-marching kernel), also inside the objective window, where the
    K-step launches accumulate the Nusselt sums themselves; J and the
    gradients are bitwise those of single-step launches, with a window
    length that is not a multiple of K and a cavity wider than one tile."""
    from paper_1601_04633_amd.dmrt import Cavity
    n, N, K, C = 70, 401, 149, 64
    tw = inputs.hot_wall_profile(n, 29)
    t0 = inputs.theta_noise(n, 30, amp=1e-2)
    out = []
    for temporal in ((1, 10), (2, 6), (2, 16), (3, 10), (3, 12), (4, 12), (4, 16), ("march", 4, 3),
                     ("march", 3, 2, 9), ("march", 6, 2)):
        print(f"[adjoint] forward steps/launch, rows {temporal} {precision}", flush=True)
        c = Cavity(n=n, Ra=1e4, Pr=0.01, precision=precision)
        if temporal[0] == "march":
            c.set_temporal_march(*temporal[1:])
        else:
            c.set_temporal(*temporal)
        c.set_hot_wall(tw)
        c.set_theta(t0)
        out.append(c.adjoint_nu(N, K, C))
        c.close()
    for o in out[1:]:
        assert o[0] == out[0][0]
        assert np.array_equal(o[1], out[0][1]) and np.array_equal(o[2], out[0][2])


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_multi_step_backward_does_not_change_gradients(precision):
    """The backward may take K adjoint (and recompute) steps per launch
    through LDS; the gradients are bitwise those of single-step launches,
    also when the segment lengths are not multiples of K and when the
    objective window starts inside a K-step launch."""
    from paper_1601_04633_amd.dmrt import Cavity
    n, N, K, C = 70, 431, 149, 64
    tw = inputs.hot_wall_profile(n, 31)
    t0 = inputs.theta_noise(n, 32, amp=1e-2)
    out = []
    for temporal in ((1, 10), (2, 6), (2, 16), (3, 10), (3, 16), (4, 16)):
        print(f"[adjoint] backward steps/launch, rows {temporal} {precision}", flush=True)
        c = Cavity(n=n, Ra=1e4, Pr=0.01, precision=precision)
        c.adjoint_set_temporal(*temporal)
        c.set_hot_wall(tw)
        c.set_theta(t0)
        out.append(c.adjoint_nu(N, K, C))
        c.close()
    for o in out[1:]:
        assert o[0] == out[0][0]
        assert np.array_equal(o[1], out[0][1]) and np.array_equal(o[2], out[0][2])


def test_multi_step_backward_against_reference():
    """K steps per backward launch against the CPU reference gradient."""
    from oracle.torch_ref import Reference
    n, N, K, C = 32, 600, 150, 100
    tw = inputs.hot_wall_profile(n, 23)
    t0 = inputs.theta_noise(n, 24, amp=1e-2)
    c = _cavity(n, 1e4, 0.01)
    c.adjoint_set_temporal(3, 10)
    c.set_hot_wall(tw)
    c.set_theta(t0)
    Jg, gw, g0 = c.adjoint_nu(N, K, C)
    c.close()
    Jr, rw, r0 = Reference(n, 1e4, 0.01).gradient(tw, t0, N, K, segment=100)
    assert abs(Jg - Jr) <= 1e-12 * abs(Jr)
    assert rel(gw, rw) <= 1e-10 and rel(g0, r0) <= 1e-10


def test_interleaved_objectives_on_one_cavity():
    """Two objectives recorded on one cavity before one backward over their
    sum: each gets the gradient of its own forward run (bitwise those of
    separate cavities), and a hot-wall change between a forward and its
    backward does not leak into the gradient."""
    import torch
    from paper_1601_04633_amd.adjoint import nu_objective
    n, N, K, C = 24, 200, 50, 40
    tw1 = torch.tensor(inputs.hot_wall_profile(n, 41), requires_grad=True)
    t01 = torch.tensor(inputs.theta_noise(n, 42, amp=1e-2), requires_grad=True)
    tw2 = torch.tensor(inputs.hot_wall_profile(n, 43, amp=3e-2), requires_grad=True)
    t02 = torch.tensor(inputs.theta_noise(n, 44, amp=2e-2), requires_grad=True)
    c = _cavity(n, 1e4, 0.01)
    J1 = nu_objective(tw1, t01, c, N, K, C)
    J2 = nu_objective(tw2, t02, c, N, K, C)
    (J1 + 3.0 * J2).backward()
    r1 = _gpu_grad(n, 1e4, 0.01, tw1.detach().numpy(), t01.detach().numpy(), N, K, C)
    r2 = _gpu_grad(n, 1e4, 0.01, tw2.detach().numpy(), t02.detach().numpy(), N, K, C)
    assert float(J1.detach()) == r1[0] and float(J2.detach()) == r2[0]
    assert np.array_equal(tw1.grad.numpy(), r1[1]) and np.array_equal(t01.grad.numpy(), r1[2])
    assert np.array_equal(tw2.grad.numpy(), 3.0 * r2[1]) and np.array_equal(t02.grad.numpy(), 3.0 * r2[2])
    # a wall change between forward and backward
    tw3 = torch.tensor(inputs.hot_wall_profile(n, 45), requires_grad=True)
    J3 = nu_objective(tw3, t01.detach().clone(), c, N, K, C)
    c.set_hot_wall(inputs.hot_wall_profile(n, 46))
    J3.backward()
    r3 = _gpu_grad(n, 1e4, 0.01, tw3.detach().numpy(), t01.detach().numpy(), N, K, C)
    assert np.array_equal(tw3.grad.numpy(), r3[1])
    c.close()


def test_backward_refused_after_invalidating_calls():
    """dmrt_adjoint_backward is refused (EINVAL) once the wall, the initial
    field or the state has been replaced since the forward run, and the
    generation counter reports it; stepping the handle does not."""
    from paper_1601_04633_amd.dmrt import DmrtError
    n, N, K, C = 16, 40, 10, 10
    tw = inputs.hot_wall_profile(n, 47)
    t0 = inputs.theta_noise(n, 48, amp=1e-2)
    c = _cavity(n, 1e4, 0.01)
    assert c.adjoint_generation() == 0
    blob = c.save_state()
    gens = []
    for spoil in (lambda: c.set_hot_wall(tw), lambda: c.set_theta(t0), lambda: c.load_state(blob),
                  lambda: c.set_temporal(2, 6), None):
        c.set_hot_wall(tw)
        c.set_theta(t0)
        c.adjoint_forward(N, K, C)
        gens.append(c.adjoint_generation())
        if spoil is None:
            c.step(7)
            assert c.adjoint_generation() == gens[-1]
            c.adjoint_backward()
        else:
            spoil()
            assert c.adjoint_generation() == 0
            with pytest.raises(DmrtError):
                c.adjoint_backward()
    assert gens == [1, 2, 3, 4, 5]
    c.close()
