"""Packed uneven batches: contact classes per env with overflow fallback,
the persistent work queues, graph replay and the launch-plan autotuner.

Every env's result depends only on its inputs and on the kernel
instantiation (contact class) that finishes it, so the class-split launch
is checked bitwise against plain one-workgroup-per-env launches of the
matching class."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2207_06649_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2207_06649_amd import pmbs
    return pmbs


def f32(a):
    return np.asarray(a, np.float64).astype(np.float32).astype(np.float64)


def grid_env(n=16, cols=4, e=0.04):
    """n cubes on a touching grid (1 mm gaps, inside the contact margin),
    rows and columns jittered by 2-3 mm: about 64 table and 96 box-box
    contacts, more than 128 and fewer than 256."""
    st = np.zeros((n, 13))
    bd = np.zeros((n, 5))
    for k in range(n):
        i, j = divmod(k, cols)
        st[k, :3] = (i * (e + 0.001) + 0.002 * j, j * (e + 0.001) + 0.003 * i, e / 2)
        st[k, 3] = 1.0
        bd[k] = (e / 2, e / 2, e / 2, 0.1, 0.5)
    return scenes.Batch(np.array([0, n], np.int32), st, bd, np.zeros((1, 4)), np.zeros(1, np.int32))


def uneven_case(seed, n_envs, n_bodies=(5, 30), region=0.3, n_grid=0):
    rng = np.random.default_rng([seed, 7])
    b = scenes.clutter_batch(seed, n_envs, n_bodies, region=region)
    if n_grid:
        b = scenes.concat([b] + [grid_env() for _ in range(n_grid)])
        n_envs += n_grid
    h = scenes.horizons(seed, n_envs)
    acts, off = [], [0]
    for e in range(n_envs):
        nb = int(b.counts()[e])
        if e >= n_envs - n_grid:
            # into the grid from outside its corner cube (object 0, direction 4: start on its -x side)
            acts += [4] * int(h[e])
        else:
            acts += [int(rng.integers(0, nb)) * 8 + int(rng.integers(0, 8)) for _ in range(int(h[e]))]
        off.append(len(acts))
    tgt = np.array([int(rng.integers(0, int(n))) for n in b.counts()], np.int32)
    return b, np.array(acts, np.int32), np.array(off, np.int32), tgt


class Run:
    """A simulator holding the batch in pool slots 0..E-1; rollouts write
    children to slots E..2E-1."""

    def __init__(self, pm, b, max_contacts):
        import torch
        E = b.n_envs
        self.E, self.b, self.pm = E, b, pm
        self.sim = pm.Sim(max_envs=E, max_bodies=b.n_bodies, max_contacts=max_contacts, pool_slots=2 * E,
                          pool_stride=31, max_horizon=5)
        self.sim.set_state(b.env_offset, f32(b.state), f32(b.body))
        self.src = np.arange(E, dtype=np.int32)
        self.child = self.src + E
        self.sim.pool_scatter(self.src)
        self.rew = torch.zeros((E, 5), dtype=torch.float32, device="cuda:0")
        self.cnt = torch.zeros(E, dtype=torch.int32, device="cuda:0")

    def go(self, acts, off, tgt, substeps, flags):
        self.sim.rollout(acts, off, tgt, n_substeps=substeps, src_slot=self.src, child_slot=self.child, max_h=5,
                         flags=flags, rewards=self.rew, counts=self.cnt, sync=False)
        return self.result()

    def result(self):
        self.sim.sync()
        rew, cnt = self.rew.cpu().numpy().copy(), self.cnt.cpu().numpy().copy()
        status = self.sim.env_status().copy()
        self.sim.pool_gather(self.child)
        st = self.sim.get_state().copy()
        return rew, cnt, status, st


def env_equal(b, e, x, y):
    """Bitwise equality of env e's rewards, count, status and child state."""
    rx, cx, sx, stx = x
    ry, cy, sy, sty = y
    lo, hi = b.env_offset[e], b.env_offset[e + 1]
    if cx[e] != cy[e] or sx[e] != sy[e]:
        return False
    if not np.array_equal(rx[e, :cx[e]], ry[e, :cy[e]]):
        return False
    # the child slot holds a state only when the expansion push was valid
    return bool(sx[e] & 4) or np.array_equal(stx[lo:hi], sty[lo:hi])


SUB = 8


@pytest.fixture(scope="module")
def case(pm):
    b, acts, off, tgt = uneven_case(5, 92, n_grid=4)
    ref128 = Run(pm, b, 128).go(acts, off, tgt, SUB, 0)
    ref256 = Run(pm, b, 256).go(acts, off, tgt, SUB, 0)
    return b, acts, off, tgt, ref128, ref256


def test_class_split_matches_plain_launches_bitwise(pm, case):
    b, acts, off, tgt, ref128, ref256 = case
    r = Run(pm, b, 256)
    r.sim.set_launch_plan(small_max_bodies=16)
    got = r.go(acts, off, tgt, SUB, pm.ROLLOUT_QUEUE)
    nb = b.counts()
    for e in range(b.n_envs):
        small_ok = nb[e] <= 16 and not (ref128[2][e] & 1)
        assert env_equal(b, e, got, ref128 if small_ok else ref256), e


def test_contact_classes_give_identical_rollouts(pm, case):
    """An env that fits the 128-contact kernel gets bitwise the same rewards,
    status and child state from the 256-contact kernel: the result does not
    depend on the class (so neither on the autotuned class threshold)."""
    b, acts, off, tgt, ref128, ref256 = case
    fits = [e for e in range(b.n_envs) if not (ref128[2][e] & 1)]
    assert len(fits) > b.n_envs // 2
    for e in fits:
        assert env_equal(b, e, ref128, ref256), e


def test_overflow_fallback_reruns_in_the_larger_class(pm, case):
    """Every env in the 128-contact kernel: those that overflow it finish in
    the 256-contact kernel with the plain 256-contact result."""
    b, acts, off, tgt, ref128, ref256 = case
    over = np.nonzero(ref128[2] & 1)[0]
    assert len(over) > 0, "the case must overflow 128 contacts somewhere"
    assert not np.any(ref256[2] & 1)
    r = Run(pm, b, 256)
    r.sim.set_launch_plan(small_max_bodies=31)
    got = r.go(acts, off, tgt, SUB, pm.ROLLOUT_QUEUE)
    for e in range(b.n_envs):
        assert env_equal(b, e, got, ref256 if e in over else ref128), e
    assert not np.any(got[2] & 1)


def test_graph_replays_match_eager(pm, case):
    """The captured launch replayed several times, with other work and
    synchronisations between replays, and recaptured after a plan change."""
    import torch
    b, acts, off, tgt, _, _ = case
    r = Run(pm, b, 256)
    for plan in (dict(small_max_bodies=16), dict(small_max_bodies=12, small_blocks_per_cu=1, order=0)):
        r.sim.set_launch_plan(**plan)
        eager = r.go(acts, off, tgt, SUB, pm.ROLLOUT_QUEUE)
        for k in range(3):
            x = torch.randn(1 << 16, device="cuda:0")
            (x * 2).sum().item()
            r.rew.fill_(-7.0)
            r.cnt.fill_(-7)
            got = r.go(acts, off, tgt, SUB, pm.ROLLOUT_QUEUE | pm.ROLLOUT_GRAPH)
            for e in range(b.n_envs):
                assert env_equal(b, e, got, eager), (plan, k, e)


def test_autotune_installs_a_plan_and_caches_it(pm, case, tmp_path):
    b, acts, off, tgt, ref128, ref256 = case
    r = Run(pm, b, 256)
    cache = tmp_path / "tune.txt"
    plan, ms, hit = r.sim.autotune(acts, off, tgt, n_substeps=SUB, src_slot=r.src, child_slot=r.child, max_h=5,
                                   reps=1, cache_path=str(cache), rewards=r.rew, counts=r.cnt)
    assert not hit and ms > 0
    assert r.sim.launch_plan() == plan
    got = r.result()
    T = plan["small_max_bodies"]
    nb = b.counts()
    for e in range(b.n_envs):
        small_ok = nb[e] <= T and not (ref128[2][e] & 1)
        assert env_equal(b, e, got, ref128 if small_ok else ref256), e
    r2 = Run(pm, b, 256)
    plan2, ms2, hit2 = r2.sim.autotune(acts, off, tgt, n_substeps=SUB, src_slot=r2.src, child_slot=r2.child, max_h=5,
                                       reps=1, cache_path=str(cache), rewards=r2.rew, counts=r2.cnt)
    assert hit2 and plan2 == plan and abs(ms2 - ms) < 1e-3 * max(1.0, ms)


def test_packed_matches_plain_padded_per_push(pm):
    """The packed queued launch (every env in the 256-contact kernel) and the
    plain form (envs padded to 30 bodies far from the scene, one launch per
    push index, host-side rollout rules) give bitwise the same rewards and
    final states of the real bodies."""
    import bench
    b, acts, off, tgt = uneven_case(9, 40, region=0.35)
    sim = pm.Sim(max_envs=b.n_envs, max_bodies=b.n_bodies, max_contacts=256, max_horizon=5)
    sim.set_launch_plan(small_max_bodies=-1)
    sim.set_state(b.env_offset, f32(b.state), f32(b.body))
    rew, cnt = sim.rollout(acts, off, tgt, n_substeps=SUB, max_h=5,
                           flags=pm.ROLLOUT_QUEUE | pm.ROLLOUT_WRITE_STATE)
    st = sim.get_state()
    status = sim.env_status()
    pb = scenes.pad_batch(b, 30)
    psim = pm.Sim(max_envs=b.n_envs, max_bodies=pb.n_bodies, max_contacts=256, max_horizon=5)
    psim.set_state(pb.env_offset, f32(pb.state), f32(pb.body))
    prew, pcnt, pstatus = bench.plain_per_push(psim, acts, off, tgt, SUB)
    pst = psim.get_state()
    assert np.array_equal(cnt, pcnt)
    assert np.array_equal(status & 5, pstatus & 5)
    for e in range(b.n_envs):
        k = cnt[e]
        assert np.array_equal(rew[e, :k], prew[e, :k]), e
        lo, hi = b.env_offset[e], b.env_offset[e + 1]
        assert np.array_equal(st[lo:hi], pst[30 * e:30 * e + (hi - lo)]), e


def test_two_level_fallback_reaches_the_512_contact_kernel(pm):
    """A 30-cube touching grid (about 400 contacts) overflows both the 128-
    and the 256-contact kernels: with max_contacts 512 it finishes in the
    512-contact kernel, bitwise equal to a plain 512-contact launch, eagerly
    and replayed as a graph."""
    b, acts, off, tgt = uneven_case(13, 20, n_bodies=(5, 12), region=0.3, n_grid=0)
    b = scenes.concat([b, grid_env(n=30, cols=6)])
    acts = np.concatenate([acts, np.array([4, 4], np.int32)])
    off = np.concatenate([off, [off[-1] + 2]]).astype(np.int32)
    tgt = np.concatenate([tgt, [0]]).astype(np.int32)
    ref = Run(pm, b, 512).go(acts, off, tgt, SUB, 0)
    r = Run(pm, b, 512)
    r.sim.set_launch_plan(small_max_bodies=31)
    for flags in (pm.ROLLOUT_QUEUE, pm.ROLLOUT_QUEUE | pm.ROLLOUT_GRAPH, pm.ROLLOUT_QUEUE | pm.ROLLOUT_GRAPH):
        r.rew.fill_(-3.0)
        got = r.go(acts, off, tgt, SUB, flags)
        for e in range(b.n_envs):
            assert env_equal(b, e, got, ref), (flags, e)
    c128 = Run(pm, b, 128).go(acts, off, tgt, SUB, 0)
    c256 = Run(pm, b, 256).go(acts, off, tgt, SUB, 0)
    assert c128[2][-1] & 1 and c256[2][-1] & 1 and not (ref[2][-1] & 1)


def test_queued_graph_rollouts_match_the_oracle(pm):
    """64 uneven envs (5-30 cuboids, 1-5 contour pushes of 20 substeps) in the
    class-split persistent queues, replayed twice as a graph: every env's
    reward count matches the FP64 oracle's rollout of the same actions and
    its rewards agree within 1e-3 (80 um of clearance, inside the
    multi-substep state bar of 1e-3 m)."""
    b, acts, off, tgt = uneven_case(17, 64)
    subs = 20
    cfg = O.make_config()
    refs = []
    for e in range(b.n_envs):
        lo, hi = b.env_offset[e], b.env_offset[e + 1]
        od = [(int(a) // 8, int(a) % 8) for a in acts[off[e]:off[e + 1]]]
        refs.append(O.rollout(cfg, f32(b.state[lo:hi]), f32(b.body[lo:hi]), od, subs, int(tgt[e]), 0.08))
    r = Run(pm, b, 256)
    r.sim.set_launch_plan(small_max_bodies=16)
    for k in range(2):
        r.rew.fill_(-5.0)
        rew, cnt, status, _ = r.go(acts, off, tgt, subs, pm.ROLLOUT_QUEUE | pm.ROLLOUT_GRAPH)
        assert not np.any(status & 3)
        for e, ref in enumerate(refs):
            n = ref["applied"]
            assert cnt[e] == n, (k, e, cnt[e], n)
            assert np.abs(rew[e, :n] - ref["rewards"]).max(initial=0.0) <= 1e-3, (k, e, rew[e, :n], ref["rewards"])


@pytest.mark.parametrize("waves", [(2, 1), (1, 2), (2, 2)])
def test_two_wave_workgroups_are_bitwise_one_wave(pm, case, waves):
    """Two waves per environment (the second takes half the contact slots
    and every second narrowphase pass) in either class: every env's
    rewards, count, status and child state are bitwise those of one wave,
    eagerly and replayed as a graph; the two shapes also race-check each
    other's LDS hand-offs."""
    b, acts, off, tgt, ref128, ref256 = case
    r = Run(pm, b, 256)
    r.sim.set_launch_plan(small_max_bodies=16, small_waves=waves[0], large_waves=waves[1])
    nb = b.counts()
    for flags in (pm.ROLLOUT_QUEUE, pm.ROLLOUT_QUEUE | pm.ROLLOUT_GRAPH, pm.ROLLOUT_QUEUE | pm.ROLLOUT_GRAPH):
        r.rew.fill_(-2.0)
        got = r.go(acts, off, tgt, SUB, flags)
        for e in range(b.n_envs):
            small_ok = nb[e] <= 16 and not (ref128[2][e] & 1)
            assert env_equal(b, e, got, ref128 if small_ok else ref256), (waves, flags, e)


def test_two_wave_step_is_bitwise_one_wave(pm):
    """pmbs_sim_step (one workgroup per env) with two waves per env: the
    state after 40 substeps of pushed 15-cuboid clutter and the env status
    are bitwise those of one wave, in the 128- and the 256-contact class."""
    b = scenes.clutter_batch(8, 96, 15)
    for mc in (128, 256):
        out = {}
        for w in (1, 2):
            sim = pm.Sim(max_envs=b.n_envs, max_bodies=b.n_bodies, max_contacts=mc)
            sim.set_launch_plan(small_waves=w, large_waves=w)
            sim.set_state(b.env_offset, f32(b.state), f32(b.body))
            sim.step(b.push.astype(np.float32), 40)
            out[w] = (sim.get_state(), sim.env_status().copy())
        assert np.array_equal(out[1][0], out[2][0]), mc
        assert np.array_equal(out[1][1], out[2][1]), mc
