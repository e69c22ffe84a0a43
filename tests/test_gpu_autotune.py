"""The autotuner on the device: it tries every configuration of its search
spaces (tile and row-marching K-step forms, launch shapes, batch schedules,
adjoint steps per launch) without error, leaves the fastest applied, stores
it in the cache and reapplies it from there; the tuned runs give bitwise the
state of untuned ones (launch configurations change only the time)."""
import numpy as np
import pytest

from paper_1601_04633_amd import autotune, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture
def cache(tmp_path, monkeypatch):
    path = tmp_path / "tune.json"
    monkeypatch.setattr(autotune, "CACHE_PATH", str(path))
    return path


@pytest.mark.parametrize("n", [64, 300])
def test_tune_cavity_then_step_bitwise(cache, n):
    from paper_1601_04633_amd.dmrt import Cavity
    th0 = inputs.theta_noise(n, 7, amp=1e-2)
    c = Cavity(n=n, Ra=1e4, Pr=0.01, precision="fp32")
    c.set_theta(th0)
    best, t, trials = autotune.tune_cavity(c, steps=24)
    assert len(trials) >= len(autotune.CAVITY_SPACE["temporal"]) and t > 0
    assert tuple(best["temporal"]) in [tuple(x) for x in autotune.CAVITY_SPACE["temporal"]]
    c.set_theta(th0)
    c.step(97)
    f1, g1 = c.raw_state()
    c.close()
    ref = Cavity(n=n, Ra=1e4, Pr=0.01, precision="fp32")
    ref.set_theta(th0)
    ref.step(97)
    f0, g0 = ref.raw_state()
    ref.close()
    assert np.array_equal(f0, f1) and np.array_equal(g0, g1)
    # from the cache: no trials, the same configuration
    c2 = Cavity(n=n, Ra=1e4, Pr=0.01, precision="fp32")
    hit, _, trials2 = autotune.tune_cavity(c2, steps=24)
    assert trials2 == [] and list(hit["temporal"]) == list(best["temporal"])
    c2.close()


def test_tune_periodic_after_cavity_at_same_size(cache):
    """A cached cavity-mode entry (which may hold a K-step form) is not
    applied to a periodic box of the same size: each wall configuration is
    tuned and cached under its own key."""
    from paper_1601_04633_amd.dmrt import Cavity
    n = 64
    c = Cavity(n=n, Ra=1e4, Pr=0.01, precision="fp32")
    c.set_theta(inputs.theta_noise(n, 8, amp=1e-2))
    autotune.tune_cavity(c, steps=24)
    c.close()
    p = Cavity(n=n, Ra=1e4, Pr=0.01, precision="fp32", bc_mode=1, gbeta_override=1e-4)
    p.set_theta(inputs.theta_noise(n, 9, amp=1e-2))
    best, t, trials = autotune.tune_cavity(p, steps=24)
    assert trials and tuple(best["temporal"]) == (1, 10)
    p.step(10)
    p.close()


def test_tune_batch_then_step_bitwise(cache):
    from paper_1601_04633_amd.dmrt import Batch, Cavity
    members = [dict(n=40, Ra=1e4, Pr=0.01), dict(n=70, Ra=3e4, Pr=0.005)]
    b = Batch(members, precision="fp32")
    for i, m in enumerate(members):
        b.set_theta(i, inputs.theta_noise(m["n"], 20 + i, amp=1e-2))
    cfg, t, trials = autotune.tune_batch(b, min_steps=64)
    assert len(trials) > 1 and t > 0
    for i, m in enumerate(members):
        b.set_theta(i, inputs.theta_noise(m["n"], 20 + i, amp=1e-2))
    b.step(128)
    for i, m in enumerate(members):
        c = Cavity(precision="fp32", **m)
        c.set_theta(inputs.theta_noise(m["n"], 20 + i, amp=1e-2))
        c.step(128)
        f, g = c.raw_state()
        c.close()
        fb, gb = b.raw_state(i)
        assert np.array_equal(f, fb) and np.array_equal(g, gb), i
    b.close()


def test_tune_adjoint_keeps_gradients(cache):
    from paper_1601_04633_amd.dmrt import Cavity
    n = 24
    tw = inputs.hot_wall_profile(n, 3)
    t0 = inputs.theta_noise(n, 4, amp=1e-2)
    c = Cavity(n=n, Ra=1e4, Pr=0.01, precision="fp64")
    c.set_hot_wall(tw)
    c.set_theta(t0)
    best, t, trials = autotune.tune_adjoint(c, nsteps=120, avg_last=40, ckpt_every=50)
    assert len(trials) == len(autotune.ADJOINT_SPACE) and tuple(best) in autotune.ADJOINT_SPACE
    c.set_theta(t0)
    J, gw, g0 = c.adjoint_nu(120, 40, 50)
    c.close()
    r = Cavity(n=n, Ra=1e4, Pr=0.01, precision="fp64")
    r.set_hot_wall(tw)
    r.set_theta(t0)
    Jr, rw, r0 = r.adjoint_nu(120, 40, 50)
    r.close()
    assert J == Jr and np.array_equal(gw, rw) and np.array_equal(g0, r0)
