"""GPU tests of the batched sweep (many cavities, one launch per step):
every member evolves bitwise as the same cavity run alone through
dmrt_step (same precision), whatever the schedule; the FP64 members match
the oracle; per-member Nu is reduced on the device; a member whose state
turns non-finite is flagged and skipped while the others continue."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_1601_04633_amd import inputs

MEMBERS = [dict(n=64, Ra=1e4, Pr=0.01), dict(n=100, Ra=3e3, Pr=0.005),
           dict(n=37, Ra=1e5, Pr=0.001), dict(n=128, Ra=2e4, Pr=0.01),
           dict(n=256, Ra=1e5, Pr=0.005), dict(n=70, Ra=1e3, Pr=0.001)]

SCHEDULES = [
    dict(block_x=64, block_y=4, order=1, grid_blocks=0, group_bytes=0, group_steps=64),
    dict(block_x=256, block_y=1, order=0, grid_blocks=0, group_bytes=0, group_steps=64, temporal=(2, 6)),
    dict(block_x=64, block_y=4, order=2, grid_blocks=200, group_bytes=3 << 20, group_steps=7,
         temporal=(2, 10)),
    dict(block_x=128, block_y=2, order=1, grid_blocks=0, group_bytes=0, group_steps=32, temporal=(2, 16)),
    dict(block_x=256, block_y=1, order=0, grid_blocks=0, group_bytes=0, group_steps=10),
    dict(block_x=64, block_y=1, order=2, grid_blocks=300, group_bytes=0, group_steps=7),
    dict(block_x=128, block_y=2, order=1, grid_blocks=0, group_bytes=3 << 20, group_steps=16),
    dict(block_x=256, block_y=1, order=1, grid_blocks=0, group_bytes=0, group_steps=64, temporal=(3, 16)),
    dict(block_x=64, block_y=4, order=2, grid_blocks=500, group_bytes=3 << 20, group_steps=10,
         temporal=(3, 10)),
    dict(block_x=256, block_y=1, order=0, grid_blocks=0, group_bytes=0, group_steps=11, temporal=(4, 16)),
    # row-marching form: automatic chunks (one resident round), fixed short
    # chunks, cavity groups, six steps per launch, the two-step form
    dict(block_x=64, block_y=4, order=1, grid_blocks=0, group_bytes=0, group_steps=64,
         temporal=("march", 4, 3, 0)),
    dict(block_x=128, block_y=2, order=2, grid_blocks=0, group_bytes=3 << 20, group_steps=12,
         temporal=("march", 4, 2, 9)),
    dict(block_x=256, block_y=1, order=0, grid_blocks=0, group_bytes=0, group_steps=30,
         temporal=("march", 6, 2, 0)),
    dict(block_x=64, block_y=4, order=1, grid_blocks=0, group_bytes=0, group_steps=16,
         temporal=("march", 2, 8, 5)),
]


def _apply_temporal(b, temporal):
    if temporal[0] == "march":
        b.set_temporal_march(*temporal[1:])
    else:
        b.set_temporal(*temporal)


def _single(member, precision, th0, steps):
    from paper_1601_04633_amd.dmrt import Cavity
    c = Cavity(precision=precision, **member)
    c.set_theta(th0)
    c.step(steps)
    return c


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("sched", range(len(SCHEDULES)))
def test_batch_members_bitwise_equal_single(precision, sched):
    from paper_1601_04633_amd.dmrt import Batch
    print(f"[batch] {precision} schedule {SCHEDULES[sched]}", flush=True)
    b = Batch(MEMBERS, precision=precision)
    sc = dict(SCHEDULES[sched])
    temporal = sc.pop("temporal", (1, 10))
    b.set_schedule(**sc)
    _apply_temporal(b, temporal)
    th = [inputs.theta_noise(m["n"], 100 + i, amp=1e-3) for i, m in enumerate(MEMBERS)]
    for i, t in enumerate(th):
        b.set_theta(i, t)
    b.step(131)
    b.step(2)
    nu_b = b.nusselt()
    for i, m in enumerate(MEMBERS):
        c = _single(m, precision, th[i], 133)
        fb, gb = b.raw_state(i)
        fc, gc = c.raw_state()
        assert np.array_equal(fb, fc) and np.array_equal(gb, gc), (i, m)
        assert nu_b[i] == c.nusselt(0)[0]


def test_batch_fp64_member_matches_oracle(oracle_mod):
    from paper_1601_04633_amd.dmrt import Batch
    b = Batch(MEMBERS[:3], precision="fp64")
    th = [inputs.theta_noise(m["n"], 7 + i) for i, m in enumerate(MEMBERS[:3])]
    for i, t in enumerate(th):
        b.set_theta(i, t)
    b.step(120)
    for i, m in enumerate(MEMBERS[:3]):
        o = oracle_mod.Oracle(m["n"], m["Ra"], m["Pr"])
        o.set_theta(th[i])
        o.step(120)
        for a, r in zip(b.fields(i), o.fields()):
            assert np.linalg.norm(a - r) <= 1e-12 * np.linalg.norm(r)


def test_batch_hot_wall_profile():
    from paper_1601_04633_amd.dmrt import Batch, Cavity
    m = MEMBERS[0]
    b = Batch([m, MEMBERS[1]], precision="fp64")
    tw = inputs.hot_wall_profile(m["n"], 3)
    b.set_hot_wall(0, tw)
    b.set_theta(0, inputs.theta_noise(m["n"], 4))
    b.step(50)
    c = Cavity(precision="fp64", **m)
    c.set_hot_wall(tw)
    c.set_theta(inputs.theta_noise(m["n"], 4))
    c.step(50)
    assert np.array_equal(b.raw_state(0)[0], c.raw_state()[0])
    assert b.nusselt()[0] == c.nusselt(0)[0]


def test_dead_member_is_flagged_and_skipped():
    from paper_1601_04633_amd.dmrt import Batch
    b = Batch(MEMBERS[:4], precision="fp32")
    th = [inputs.theta_noise(m["n"], 20 + i) for i, m in enumerate(MEMBERS[:4])]
    for i, t in enumerate(th):
        b.set_theta(i, t)
    b.step(10)
    assert list(b.status()) == [0, 0, 0, 0]
    f, g = b.raw_state(2)
    f[3, 5, 7] = np.nan                      # planted on the host
    b.load_state(2, f, g)
    b.step(20)
    st = b.status()
    assert st[2] != 0 and st[0] == 0 and st[1] == 0 and st[3] == 0
    nu = b.nusselt()
    assert np.isnan(nu[2]) and np.all(np.isfinite(nu[[0, 1, 3]]))
    frozen = b.raw_state(2)
    b.step(30)
    # the dead member is skipped; the others match their single runs
    after = b.raw_state(2)
    assert np.array_equal(frozen[0], after[0], equal_nan=True)
    for i in (0, 1, 3):
        c = _single(MEMBERS[i], "fp32", th[i], 60)
        assert np.array_equal(b.raw_state(i)[0], c.raw_state()[0])
    # re-initialising revives it
    b.set_theta(2, th[2])
    assert b.status()[2] == 0


def test_dead_member_skipped_by_the_marching_form():
    """A member planted with NaN is flagged and skipped by the batched
    marching launches (six steps each) while the others keep matching
    their single runs bitwise."""
    from paper_1601_04633_amd.dmrt import Batch
    b = Batch(MEMBERS[:4], precision="fp32")
    b.set_temporal_march(6, 2, 0)
    th = [inputs.theta_noise(m["n"], 20 + i) for i, m in enumerate(MEMBERS[:4])]
    for i, t in enumerate(th):
        b.set_theta(i, t)
    b.step(12)
    assert list(b.status()) == [0, 0, 0, 0]
    f, g = b.raw_state(1)
    g[2, 9, 4] = np.inf                      # planted on the host
    b.load_state(1, f, g)
    b.step(24)
    st = b.status()
    assert st[1] != 0 and st[0] == 0 and st[2] == 0 and st[3] == 0
    frozen = b.raw_state(1)
    b.step(36)                               # six launches: the same copy is current again
    after = b.raw_state(1)
    assert np.array_equal(frozen[0], after[0], equal_nan=True)
    assert np.array_equal(frozen[1], after[1], equal_nan=True)
    for i in (0, 2, 3):
        c = _single(MEMBERS[i], "fp32", th[i], 72)
        assert np.array_equal(b.raw_state(i)[0], c.raw_state()[0]), i
        assert np.array_equal(b.raw_state(i)[1], c.raw_state()[1]), i


def test_sweep_shaped_batch_sampled_members():
    """The 64-cavity sweep (sides 64..512, Ra 1e3..1e5, Pr 0.001..0.01, FP32)
    in the default schedule: sampled members equal their single runs."""
    from paper_1601_04633_amd.dmrt import Batch
    specs = inputs.batch_cavities(64, 4633)
    members = [dict(n=s, Ra=ra, Pr=pr) for s, ra, pr in specs]
    b = Batch(members, precision="fp32")
    th = {}
    for i, m in enumerate(members):
        th[i] = inputs.theta_noise(m["n"], 4633 + i)
        b.set_theta(i, th[i])
    b.step(200)
    nu = b.nusselt()
    assert np.all(np.isfinite(nu))
    sides = [m["n"] for m in members]
    picks = {sides.index(s) for s in set(sides)}
    for i in sorted(picks):
        c = _single(members[i], "fp32", th[i], 200)
        assert np.array_equal(b.raw_state(i)[0], c.raw_state()[0]), i
        assert nu[i] == c.nusselt(0)[0]


@pytest.mark.parametrize("temporal", [(1, 10), (2, 6), (4, 16), ("march", 4, 3, 0), ("march", 6, 2, 3)])
def test_tiny_and_ragged_members_bitwise_equal_single(temporal):
    """Members smaller than one footprint (4^2, 5^2) and ragged sizes beside
    a larger one, K steps per launch: every member equals its single run."""
    from paper_1601_04633_amd.dmrt import Batch
    members = [dict(n=4, Ra=1e4, Pr=0.01), dict(n=5, Ra=3e3, Pr=0.005), dict(n=59, Ra=1e4, Pr=0.01),
               dict(n=131, Ra=5e4, Pr=0.005)]
    b = Batch(members, precision="fp32")
    _apply_temporal(b, temporal)
    th = [inputs.theta_noise(m["n"], 70 + i, amp=1e-2) for i, m in enumerate(members)]
    for i, t in enumerate(th):
        b.set_theta(i, t)
    b.step(77)
    for i, m in enumerate(members):
        c = _single(m, "fp32", th[i], 77)
        fb, gb = b.raw_state(i)
        fc, gc = c.raw_state()
        assert np.array_equal(fb, fc) and np.array_equal(gb, gc), (i, m, temporal)
    assert (b.status() == 0).all()


def test_sweep_in_benchmark_schedule_sampled_members():
    """The 64-cavity sweep in a schedule of the kind the benchmark's tuner
    picks (four steps per launch on 64 x 16 footprints, a persistent grid of
    16,384 workgroups, 224 MB cavity groups of 32 steps): sampled members of
    every side equal their single runs bitwise."""
    from paper_1601_04633_amd.dmrt import Batch
    specs = inputs.batch_cavities(64, 4633)
    members = [dict(n=s, Ra=ra, Pr=pr) for s, ra, pr in specs]
    b = Batch(members, precision="fp32")
    b.set_schedule(block_x=128, block_y=2, order=1, grid_blocks=16384, group_bytes=224 << 20,
                   group_steps=32)
    b.set_temporal(4, 16)
    th = {}
    for i, m in enumerate(members):
        th[i] = inputs.theta_noise(m["n"], 4633 + i)
        b.set_theta(i, th[i])
    b.step(224)
    nu = b.nusselt()
    assert np.all(np.isfinite(nu))
    sides = [m["n"] for m in members]
    picks = {sides.index(s) for s in set(sides)} | {len(members) - 1}
    for i in sorted(picks):
        c = _single(members[i], "fp32", th[i], 224)
        assert np.array_equal(b.raw_state(i)[0], c.raw_state()[0]), i
        assert nu[i] == c.nusselt(0)[0]


@pytest.mark.parametrize("temporal", [("march", 4, 3, 0), ("march", 6, 2, 0)])
def test_sweep_in_marching_schedule_sampled_members(temporal):
    """The 64-cavity sweep with the row-marching form (every member's bands
    and chunks in one launch per group, 224 MB groups of 32 steps): sampled
    members of every side equal their single runs bitwise."""
    from paper_1601_04633_amd.dmrt import Batch
    specs = inputs.batch_cavities(64, 4633)
    members = [dict(n=s, Ra=ra, Pr=pr) for s, ra, pr in specs]
    b = Batch(members, precision="fp32")
    b.set_schedule(block_x=256, block_y=1, order=1, grid_blocks=0, group_bytes=224 << 20, group_steps=32)
    _apply_temporal(b, temporal)
    th = {}
    for i, m in enumerate(members):
        th[i] = inputs.theta_noise(m["n"], 4633 + i)
        b.set_theta(i, th[i])
    b.step(96)
    nu = b.nusselt()
    assert np.all(np.isfinite(nu))
    sides = [m["n"] for m in members]
    picks = {sides.index(s) for s in set(sides)} | {len(members) - 1}
    for i in sorted(picks):
        c = _single(members[i], "fp32", th[i], 96)
        assert np.array_equal(b.raw_state(i)[0], c.raw_state()[0]), (i, temporal)
        assert np.array_equal(b.raw_state(i)[1], c.raw_state()[1]), (i, temporal)
        assert nu[i] == c.nusselt(0)[0]
