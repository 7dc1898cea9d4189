"""GPU parity of the push transition: libpmbs (FP32, HIP) against the FP64
oracle on the same seeded inputs.

Bars (written per test): 1 substep <= 1e-5 m position and <= 1e-5
quaternion; 240 substeps <= 1e-3 m on contact-free and resting scenes;
chaotic clutter over many substeps: penetration <= 1 mm (measured by the
oracle's narrowphase on the GPU state), no NaN, no contact overflow.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2207_06649_amd import scenes

pytestmark = pytest.mark.gpu

CFG = O.make_config()
FAR = np.array([5.0, 5.0, 5.1, 5.0])


@pytest.fixture(scope="module")
def pm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2207_06649_amd import pmbs
    return pmbs


def f32(a):
    """Round inputs to float32 so both sides start from identical values."""
    return np.asarray(a, np.float64).astype(np.float32).astype(np.float64)


def qerr(a, b):
    return np.minimum(np.linalg.norm(a - b, axis=-1), np.linalg.norm(a + b, axis=-1))


def run_gpu(pm, batch, push, n_sub, **cfg):
    sim = pm.Sim(max_envs=max(batch.n_envs, 1), max_bodies=max(batch.n_bodies, 1), **cfg)
    sim.set_state(batch.env_offset, f32(batch.state), f32(batch.body))
    sim.step(np.asarray(push, np.float32).reshape(-1, 4), n_sub)
    st = sim.get_state().astype(np.float64)
    return st, sim.env_status(), sim


def run_oracle(batch, push, n_sub, threads=8):
    st, status, valid = O.step(CFG, batch.env_offset, f32(batch.state), f32(batch.body),
                               f32(np.asarray(push).reshape(-1, 4)), n_sub, n_threads=threads)
    return st, status, valid


def compare(g, o, pos_tol, q_tol, v_tol):
    """Position (m), quaternion and velocity bars.  Velocities: linear (m/s)
    and angular (rad/s) per body, both under v_tol.  After one substep the
    position bar alone would allow v errors of pos_tol / dt (2.4e-3 m/s),
    so the velocity bar is set tighter (1e-4); over 240 substeps it is the
    position bar over the 1 s simulated (1e-3)."""
    dp = np.linalg.norm(g[:, :3] - o[:, :3], axis=1).max()
    dq = qerr(g[:, 3:7], o[:, 3:7]).max()
    dv = np.linalg.norm(g[:, 7:10] - o[:, 7:10], axis=1).max()
    dw = np.linalg.norm(g[:, 10:13] - o[:, 10:13], axis=1).max()
    assert dp <= pos_tol, f"position error {dp:.3e} > {pos_tol}"
    assert dq <= q_tol, f"quaternion error {dq:.3e} > {q_tol}"
    assert dv <= v_tol, f"linear velocity error {dv:.3e} > {v_tol}"
    assert dw <= v_tol, f"angular velocity error {dw:.3e} > {v_tol}"
    return dp, dq


def touching_push(b, gap=5e-4):
    """The plain push moved forward until the pusher is `gap` from cube 0."""
    push = b.push.copy()
    h = np.array([0.01, 0.01, 0.02])

    def sep(shift):
        x = np.array([push[0, 0] + shift, push[0, 1], 0.022])
        return O.sat_max_separation(CFG, b.state[0, :3], b.state[0, 3:7], b.body[0, :3], x,
                                    np.array([1.0, 0, 0, 0]), h)

    lo, hi = 0.0, 0.06
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if sep(mid) > gap:
            lo = mid
        else:
            hi = mid
    push[0, 0] += lo
    push[0, 2] += lo
    return push


def single(state_rows, body_rows):
    st = np.atleast_2d(np.asarray(state_rows, float))
    bd = np.atleast_2d(np.asarray(body_rows, float))
    return scenes.Batch(np.array([0, len(st)], np.int32), st, bd, FAR[None].copy(), np.zeros(1, np.int32))


def srow(x, q=(1, 0, 0, 0), v=(0, 0, 0), w=(0, 0, 0)):
    return np.array([*x, *q, *v, *w], float)


# ------------------------------------------------------------- contact-free
@pytest.mark.parametrize("n_sub,tol", [(1, 1e-5), (240, 1e-3)])
def test_ballistic_and_spin(pm, n_sub, tol):
    b = single([srow((0.01, 0.02, 10.0), v=(0.3, -0.2, 0.5)),
                srow((1.0, 0.0, 12.0), q=(math.cos(0.3), math.sin(0.3), 0, 0), w=(3.0, -1.0, 2.0))],
               [[0.02, 0.02, 0.02, 0.1, 0.5], [0.03, 0.02, 0.01, 0.2, 0.4]])
    g, status, _ = run_gpu(pm, b, FAR, n_sub)
    o, _, _ = run_oracle(b, FAR, n_sub)
    compare(g, o, tol, tol, 1e-4 if n_sub == 1 else tol)
    assert status[0] == 0


# ------------------------------------------------------------- resting
@pytest.mark.parametrize("n_sub,tol", [(1, 1e-5), (240, 1e-3)])
def test_resting_boxes(pm, n_sub, tol):
    b = scenes.clutter_batch(21, 1, 12)
    g, status, _ = run_gpu(pm, b, FAR, n_sub)
    o, _, _ = run_oracle(b, FAR, n_sub)
    compare(g, o, tol, tol, 1e-4 if n_sub == 1 else tol)
    assert status[0] == 0


# ------------------------------------------------------------- narrowphase
def _contacts_match(gc, oc, tol=2e-5):
    """Same multiset of (a, b) pairs with matching points / normals / sep."""
    assert len(gc) == len(oc), (len(gc), len(oc))
    key = lambda c: (c[0], c[1], round(c[2], 3), round(c[3], 3), round(c[4], 3))
    gs, os_ = sorted(gc.tolist(), key=key), sorted(oc.tolist(), key=key)
    for x, y in zip(gs, os_):
        assert x[0] == y[0] and x[1] == y[1]
        assert np.abs(np.array(x[2:]) - np.array(y[2:])).max() < tol, (x, y)


@pytest.mark.parametrize("seed", range(6))
def test_contact_lists_plain_push_scene(pm, seed):
    """Pusher placed at its start pose and then 3 cm further, touching cube 0."""
    b = scenes.plain_push_scene(seed)
    for push in (b.push.copy(), touching_push(b)):
        sim = pm.Sim(max_envs=1, max_bodies=8)
        sim.set_state(b.env_offset, f32(b.state), f32(b.body))
        counts, contacts = sim.collide(push.astype(np.float32))
        oc, _ = O.collide(CFG, f32(b.state), f32(b.body), f32(push[0]))
        _contacts_match(contacts[0, : counts[0]], oc)


def test_contact_lists_touching_pairs(pm):
    """Face-face partial overlap, crossed edges and tilted boxes."""
    qx = (math.cos(math.pi / 8), math.sin(math.pi / 8), 0, 0)
    qy = (math.cos(math.pi / 8), 0, math.sin(math.pi / 8), 0)
    ra = math.sqrt(2) * 0.01
    cases = [
        ([srow((0, 0, 0.5)), srow((0.04 - 5e-4, 0.0011, 0.5031))],
         [[0.02, 0.03, 0.01, 0.1, 0.5], [0.02, 0.01, 0.03, 0.1, 0.5]]),
        ([srow((0.003, -0.002, 0.5), q=qx), srow((0.0, 0.0, 0.5 + 2 * ra - 6e-4), q=qy)],
         [[0.04, 0.01, 0.01, 0.1, 0.5], [0.01, 0.04, 0.01, 0.1, 0.5]]),
        ([srow((0, 0, 0.0235), q=(math.cos(0.2), 0.05, 0.0, math.sin(0.2))), srow((0.05, 0.01, 0.019))],
         [[0.025, 0.02, 0.025, 0.1, 0.5], [0.025, 0.025, 0.02, 0.1, 0.5]]),
    ]
    for st, bd in cases:
        st = np.array(st)
        st[:, 3:7] /= np.linalg.norm(st[:, 3:7], axis=1, keepdims=True)
        b = single(st, bd)
        sim = pm.Sim(max_envs=1, max_bodies=4)
        sim.set_state(b.env_offset, f32(b.state), f32(b.body))
        counts, contacts = sim.collide(None)
        oc, _ = O.collide(CFG, f32(b.state), f32(b.body))
        assert len(oc) > 0
        _contacts_match(contacts[0, : counts[0]], oc)


def test_contact_lists_batched_clutter(pm):
    b = scenes.clutter_batch(1, 64, (5, 30))
    sim = pm.Sim(max_envs=b.n_envs, max_bodies=b.n_bodies, max_contacts=512)
    sim.set_state(b.env_offset, f32(b.state), f32(b.body))
    counts, contacts = sim.collide(b.push.astype(np.float32))
    for e in range(b.n_envs):
        be = b.env(e)
        oc, _ = O.collide(CFG, f32(be.state), f32(be.body), f32(be.push[0]))
        _contacts_match(contacts[e, : counts[e]], oc)


# ------------------------------------------------------------- pushes
@pytest.mark.parametrize("seed", range(4))
def test_plain_push_one_substep(pm, seed):
    b = scenes.plain_push_scene(seed)
    # the pusher starts 0.5 mm from cube 0, so the first substep has pusher contacts
    push = touching_push(b)
    g, gs, _ = run_gpu(pm, b, push, 1)
    o, os_, ov = run_oracle(b, push, 1)
    compare(g, o, 1e-5, 1e-5, 1e-4)
    assert ov[0] == 1 and gs[0] == 0
    oc, _ = O.collide(CFG, f32(b.state), f32(b.body), f32(push[0]))
    assert np.any(oc[:, 1] == 5)


@pytest.mark.parametrize("seed", range(4))
def test_plain_push_full_invariants(pm, seed):
    """240 substeps (10 cm push): the pushed cube moves like the oracle's within
    1 mm-scale chaos bounds; penetration <= 1 mm; no NaN or overflow."""
    b = scenes.plain_push_scene(seed)
    g, gs, _ = run_gpu(pm, b, b.push, 240)
    o, os_, ov = run_oracle(b, b.push, 240)
    assert gs[0] == 0 and ov[0] == 1
    c, _ = O.collide(CFG, g, b.body)
    pen = max(0.0, -c[:, 8].min()) if len(c) else 0.0
    assert pen <= 1e-3
    assert np.isfinite(g).all()
    dx_g, dx_o = g[0, 0] - b.state[0, 0], o[0, 0] - b.state[0, 0]
    assert 0.05 < dx_g < 0.10
    assert abs(dx_g - dx_o) < 5e-3


@pytest.mark.parametrize("seed,n_sub", [(0, 20), (1, 40), (2, 40), (3, 60)])
def test_contact_onset_short_push(pm, seed, n_sub):
    """The pusher starts 3 mm from cube 0 and reaches it after about seven
    substeps: the contact list first stays unchanged (resting plane contacts,
    so incidence lists and the min-x order carry over between substeps),
    then changes at the onset and stays again.  Over this short window the
    FP32 path stays within rounding of the FP64 oracle (about 1e-8 m and
    1e-7 measured), so the bar is the one-substep bar, 1e-5 m and 1e-5; a
    stale list or order would exceed it by orders of magnitude."""
    b = scenes.plain_push_scene(seed)
    push = touching_push(b, gap=3e-3)
    g, gs, _ = run_gpu(pm, b, push, n_sub)
    o, os_, ov = run_oracle(b, push, n_sub)
    assert gs[0] == 0 and ov[0] == 1
    compare(g, o, 1e-5, 1e-5, 1e-4)
    # the push reached cube 0: it moved along the push
    assert g[0, 0] - b.state[0, 0] > 1e-4


@pytest.mark.parametrize("n_sub", [20, 40, 60])
def test_box_box_onset_short_push(pm, n_sub):
    """Two cubes in a row, 3 mm apart, and the pusher 3 mm behind the first:
    the pusher reaches cube A after about seven substeps and A reaches cube
    B a few substeps later, so face-face clipping between the cubes starts
    mid-push and the contact list changes twice.  The FP32 path stays within
    rounding of the FP64 oracle (about 1e-8 m measured): bar 1e-5 m, 1e-5."""
    h = 0.02
    b = single([srow((0.0, 0.0, h)), srow((2 * h + 3e-3, 0.0, h))],
               [[h, h, h, 0.1, 0.5], [h, h, h, 0.1, 0.5]])
    x0 = -h - 0.01 - 3e-3
    push = np.array([[x0, 0.0, x0 + 0.05, 0.0]])
    g, gs, _ = run_gpu(pm, b, push, n_sub)
    o, os_, ov = run_oracle(b, push, n_sub)
    assert gs[0] == 0 and ov[0] == 1
    compare(g, o, 1e-5, 1e-5, 1e-4)
    # both cubes were pushed: A by the pusher, B by A
    assert g[0, 0] > 1e-3 and g[1, 0] - (2 * h + 3e-3) > 1e-3


def test_invalid_push_discarded(pm):
    b = scenes.plain_push_scene(4)
    c0 = b.state[0, :2]
    bad = np.array([[c0[0], c0[1], c0[0] + 0.05, c0[1]]])
    g, gs, _ = run_gpu(pm, b, bad, 10)
    o, _, ov = run_oracle(b, bad, 10)
    assert gs[0] & 4 and ov[0] == 0
    compare(g, o, 1e-5, 1e-5, 1e-4)


# ------------------------------------------------------------- batched clutter
def test_batched_clutter_one_substep(pm):
    """1024 envs x 15 cuboids, circle pushes: every env within 1e-5 after 1 substep."""
    b = scenes.clutter_batch(1, 1024, 15)
    g, gs, _ = run_gpu(pm, b, b.push, 1)
    o, _, ov = run_oracle(b, b.push, 1)
    compare(g, o, 1e-5, 1e-5, 1e-4)
    assert np.array_equal((gs & 4) == 0, ov == 1)


def test_uneven_clutter_one_substep(pm):
    """Packed uneven envs (5-30 bodies) with 512-contact slots."""
    b = scenes.clutter_batch(3, 256, (5, 30))
    g, gs, _ = run_gpu(pm, b, b.push, 1, max_contacts=512)
    o, _, ov = run_oracle(b, b.push, 1)
    compare(g, o, 1e-5, 1e-5, 1e-4)
    assert np.array_equal((gs & 4) == 0, ov == 1)


def test_batched_clutter_120_substeps_invariants(pm):
    b = scenes.clutter_batch(1, 1024, 15)
    g, gs, _ = run_gpu(pm, b, b.push, 120)
    assert np.isfinite(g).all()
    assert not np.any(gs & 3)
    rng = np.random.default_rng(0)
    for e in rng.choice(b.n_envs, 48, replace=False):
        lo, hi = b.env_offset[e], b.env_offset[e + 1]
        c, _ = O.collide(CFG, g[lo:hi], b.body[lo:hi])
        pen = max(0.0, -c[:, 8].min()) if len(c) else 0.0
        assert pen <= 1e-3, (e, pen)


def test_clutter_settle_energy(pm):
    """48 clutter envs (15 cuboids): a 120-substep push, then a settle of 120
    substeps with the pusher parked far away (one warm-started settle: the
    state after k settle substeps is the output of a k-substep call from the
    post-push state).  Friction and inelastic contacts only remove energy;
    the Baumgarte term lifts a penetrating body by at most beta (pen - slop)
    per substep; the warm-started 10-iteration solve is not converged and
    its warm-start impulses can do positive work in a substep where a
    contact set changes (the FP64 oracle shows up to 3.4e-5 J per substep on
    these scenes, 1.2e-6 J at 30 iterations, none at 100).  Bars: every
    settle substep raises an env's energy by at most 1e-4 J plus the
    Baumgarte allowance sum_i m_i g beta (pen_i - slop)+ (penetration from
    the oracle's narrowphase on the GPU state); every env ends the settle
    with less energy than it started with; penetration <= 1 mm
    throughout."""
    b = scenes.clutter_batch(1, 48, 15)
    sim = pm.Sim(max_envs=b.n_envs, max_bodies=b.n_bodies)
    sim.set_state(b.env_offset, f32(b.state), f32(b.body))
    sim.step(b.push.astype(np.float32), 120)
    assert not np.any(sim.env_status() & 3)
    post = sim.get_state().copy()
    far = np.tile(FAR, (b.n_envs, 1)).astype(np.float32)
    beta, slop, grav, ws = 0.2, 0.0005, 9.81, 1e-4

    def energy_and_allowance(g):
        E, allow = np.zeros(b.n_envs), np.full(b.n_envs, ws)
        for e in range(b.n_envs):
            lo, hi = b.env_offset[e], b.env_offset[e + 1]
            E[e] = O.energy(CFG, g[lo:hi], b.body[lo:hi])
            c, _ = O.collide(CFG, g[lo:hi], b.body[lo:hi])
            for i in range(hi - lo):
                sel = c[(c[:, 0] == i) | (c[:, 1] == i)]
                if len(sel):
                    pen = -sel[:, 8].min()
                    assert pen <= 1e-3, (e, i, pen)
                    allow[e] += b.body[lo + i, 3] * grav * beta * max(0.0, pen - slop)
        return E, allow

    E0, allow = energy_and_allowance(post.astype(np.float64))
    E = E0
    for k in range(1, 121):
        sim.set_state(b.env_offset, post, f32(b.body))
        sim.step(far, k)
        g = sim.get_state().astype(np.float64)
        assert np.isfinite(g).all() and not np.any(sim.env_status() & 3)
        E1, allow1 = energy_and_allowance(g)
        rise = E1 - (E + allow)
        assert rise.max() <= 0.0, (k, int(rise.argmax()), rise.max())
        E, allow = E1, allow1
    assert np.all(E < E0), (E - E0).max()


def touching_cubes(layout, h=0.02, mass=0.1, mu=0.5):
    """Equal cubes on the table with faces touching: "grid" is a 3 x 3 block
    (the centre cube has 36 contacts), "rows" is 17 cubes, five rows of three
    and a pair (a middle cube has 12): lists longer than the register-held
    entries of the per-body sums."""
    if layout == "grid":
        xy = [((i - 1) * 2 * h, (j - 1) * 2 * h) for i in range(3) for j in range(3)]
    else:
        xy = [(k * 8 * h + d * 2 * h, 0.0) for k in range(5) for d in range(3)] + [(0.0, 6 * h), (2 * h, 6 * h)]
    rows = [srow((x, y, h)) for x, y in xy]
    return single(rows, [[h, h, h, mass, mu]] * len(rows))


@pytest.mark.parametrize("layout,mc", [("grid", 128), ("rows", 128)])
def test_long_incidence_lists(pm, layout, mc):
    """Per-body sums over lists longer than the register-held entries: 9
    cubes (one wave sums on lane pairs) and 17 cubes (one wave sums on
    single lanes, more than 16 cuboids).  One substep matches the oracle to
    the one-substep bars, and twenty substeps are bitwise the same with one
    and with two waves per environment (lane pairs on both waves)."""
    b = touching_cubes(layout)
    c, _ = O.collide(CFG, f32(b.state), f32(b.body))
    assert len(c) <= mc
    per_body = np.bincount(np.concatenate([c[c[:, 0] >= 0, 0], c[:, 1]]).astype(int), minlength=b.n_bodies)
    assert per_body.max() > 8, per_body
    g, status, _ = run_gpu(pm, b, FAR, 1, max_contacts=mc)
    o, _, _ = run_oracle(b, FAR, 1)
    compare(g, o, 1e-5, 1e-5, 1e-4)
    assert status[0] == 0
    out = {}
    for w in (1, 2):
        sim = pm.Sim(max_envs=1, max_bodies=b.n_bodies, max_contacts=mc)
        sim.set_launch_plan(small_waves=w, large_waves=w)
        sim.set_state(b.env_offset, f32(b.state), f32(b.body))
        sim.step(FAR.astype(np.float32).reshape(1, 4), 20)
        out[w] = (sim.get_state(), sim.env_status().copy())
    assert np.array_equal(out[1][0], out[2][0]) and np.array_equal(out[1][1], out[2][1])
    assert out[1][1][0] == 0


def test_two_waves_bitwise_on_many_touching_scenes(pm):
    """Both waves of an env run narrowphase passes with live face pairs at
    once (touching cubes, pushed into): each wave's candidate axes and clip
    polygons live in its own LDS region, so 512 such envs in one launch give
    bitwise the results of one wave per env (a shared region raced here)."""
    parts = []
    rng = np.random.default_rng(11)
    for k in range(512):
        b = touching_cubes("grid" if k % 2 == 0 else "rows")
        # a push from outside the first cube's -x face toward it, offset in y
        y = b.state[0, 1] + rng.uniform(-0.015, 0.015)
        x0 = b.state[0, 0] - 0.02 - 0.016
        b = scenes.Batch(b.env_offset, b.state, b.body, np.array([[x0, y, x0 + 0.05, y]]), b.target)
        parts.append(b)
    b = scenes.concat(parts)
    out = []
    for w in (1, 2):
        sim = pm.Sim(max_envs=b.n_envs, max_bodies=b.n_bodies, max_contacts=256)
        sim.set_launch_plan(small_waves=w, large_waves=w)
        sim.set_state(b.env_offset, f32(b.state), f32(b.body))
        sim.step(b.push.astype(np.float32), 20)
        out.append((sim.get_state(), sim.env_status().copy(), sim.stats()))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    assert np.array_equal(out[0][2], out[1][2])
    assert out[0][2][:, 1].sum() > 512 * 20 * 8   # many candidate pairs per substep


def test_contact_capacity_classes_agree(pm):
    """The 128-, 256- and 512-contact kernels run the same algorithm in the
    same order, and multiply-adds are fused only where the source says so,
    so an environment's result does not depend on the class that ran it:
    bitwise equal states and status words, after 1 and after 40 pushed
    substeps."""
    b = scenes.clutter_batch(12, 64, 15)
    for n_sub in (1, 40):
        outs = []
        for cap in (128, 256, 512):
            g, gs, _ = run_gpu(pm, b, b.push, n_sub, max_contacts=cap)
            assert not np.any(gs & 1)
            outs.append((g, gs.copy()))
        for o, os_ in outs[1:]:
            assert np.array_equal(o, outs[0][0]) and np.array_equal(os_, outs[0][1])


def grid_pile(n=31, e=0.04):
    """n cubes on a touching grid, rows and columns jittered by 2-3 mm so no
    corners coincide: far more than 128 contacts."""
    st, bd = [], []
    for k in range(n):
        i, j = divmod(k, 6)
        st.append(srow((i * e + 0.002 * j, j * e + 0.003 * i, e / 2)))
        bd.append([e / 2, e / 2, e / 2, 0.1, 0.5])
    return single(st, bd)


def test_contact_overflow_flagged_and_isolated(pm):
    """An env whose contacts exceed the cap is flagged and truncated exactly
    like the oracle's list; the other envs are bitwise what they are alone."""
    pile = grid_pile()
    small = scenes.clutter_batch(14, 3, 6)
    both = scenes.concat([pile, small])
    push = np.concatenate([FAR[None], small.push])
    g, gs, _ = run_gpu(pm, both, push, 1, max_contacts=128)
    assert gs[0] & 1 and not np.any(gs[1:] & 1)
    cfg128 = O.make_config(max_contacts=128)
    o, os_, _ = O.step(cfg128, pile.env_offset, f32(pile.state), f32(pile.body), f32(FAR[None]), 1)
    assert os_[0] & 1
    compare(g[:31], o, 1e-5, 1e-5, 1e-4)
    alone, _, _ = run_gpu(pm, small, small.push, 1, max_contacts=128)
    assert np.array_equal(g[31:], alone)


def test_headline_shape_sampled_parity(pm):
    """4096 envs x 15 cuboids in one launch (the benchmark's shape): sampled
    envs match the oracle after 1 substep; 120 substeps keep the invariants."""
    b = scenes.clutter_batch(2, 4096, 15)
    sim = pm.Sim(max_envs=b.n_envs, max_bodies=b.n_bodies)
    sim.set_state(b.env_offset, f32(b.state), f32(b.body))
    sim.step(b.push.astype(np.float32), 1)
    g = sim.get_state().astype(np.float64)
    rng = np.random.default_rng(1)
    for e in rng.choice(b.n_envs, 64, replace=False):
        be = b.env(e)
        o, _, _ = run_oracle(be, be.push, 1, threads=1)
        lo, hi = b.env_offset[e], b.env_offset[e + 1]
        compare(g[lo:hi], o, 1e-5, 1e-5, 1e-4)
    sim.set_state(b.env_offset, f32(b.state), f32(b.body))
    sim.step(b.push.astype(np.float32), 120)
    g = sim.get_state().astype(np.float64)
    st = sim.env_status()
    assert np.isfinite(g).all() and not np.any(st & 3)
    # penetration (the oracle's FP64 narrowphase on the GPU state) <= 1 mm
    for e in rng.choice(b.n_envs, 64, replace=False):
        lo, hi = b.env_offset[e], b.env_offset[e + 1]
        c, _ = O.collide(CFG, g[lo:hi], b.body[lo:hi])
        pen = max(0.0, -c[:, 8].min()) if len(c) else 0.0
        assert pen <= 1e-3, (e, pen)


def test_work_ordered_step_bitwise(pm):
    """With more envs than resident workgroups a step runs a cost pass and
    takes the envs from a queue, largest work estimate first: every env's
    result (state, status, contact statistics) is bitwise that of the plain
    launch, at the benchmark's shape and on an uneven batch in the
    256-contact class, with one and two waves per env."""
    cases = ((scenes.clutter_batch(2, 4096, 15), 128, 30), (scenes.clutter_batch(6, 2400, (5, 30)), 256, 20))
    for b, mc, n_sub in cases:
        sim = pm.Sim(max_envs=b.n_envs, max_bodies=b.n_bodies, max_contacts=mc)
        out = []
        for order, waves in ((0, 1), (1, 1), (1, 2)):
            sim.set_launch_plan(order=order, small_waves=waves, large_waves=waves)
            sim.set_state(b.env_offset, f32(b.state), f32(b.body))
            sim.step(b.push.astype(np.float32), n_sub)
            out.append((sim.get_state(), sim.env_status(), sim.stats()))
        for g, st, stats in out[1:]:
            assert np.array_equal(g, out[0][0]) and np.array_equal(st, out[0][1])
            assert np.array_equal(stats, out[0][2])


# ------------------------------------------------------------- determinism / packing
def test_run_twice_bitwise_and_alone_vs_packed(pm):
    b = scenes.clutter_batch(5, 96, (5, 30))
    g1, _, _ = run_gpu(pm, b, b.push, 60, max_contacts=512)
    g2, _, _ = run_gpu(pm, b, b.push, 60, max_contacts=512)
    assert np.array_equal(g1, g2)
    for e in (0, 17, 95):
        be = b.env(e)
        ga, _, _ = run_gpu(pm, be, be.push, 60, max_contacts=512)
        lo, hi = b.env_offset[e], b.env_offset[e + 1]
        assert np.array_equal(ga, g1[lo:hi])


# ------------------------------------------------------------- reward
def test_reward_matches_oracle(pm):
    b = scenes.clutter_batch(9, 128, (2, 30))
    tgt = np.random.default_rng(2).integers(0, 2, size=b.n_envs).astype(np.int32)
    # perturb orientations so footprints are tilted hexagons too
    st = b.state.copy()
    rng = np.random.default_rng(4)
    for i in range(0, b.n_bodies, 3):
        q = st[i, 3:7] + rng.normal(scale=0.1, size=4)
        st[i, 3:7] = q / np.linalg.norm(q)
    b2 = scenes.Batch(b.env_offset, st, b.body, b.push, tgt)
    sim = pm.Sim(max_envs=b.n_envs, max_bodies=b.n_bodies)
    sim.set_state(b2.env_offset, f32(st), f32(b.body))
    rew, clr = sim.eval_reward(tgt, 0.08)
    for e in range(b.n_envs):
        lo, hi = b.env_offset[e], b.env_offset[e + 1]
        oc = O.clearance(f32(st[lo:hi]), f32(b.body[lo:hi]), int(tgt[e]))
        orw = O.reward(f32(st[lo:hi]), f32(b.body[lo:hi]), int(tgt[e]), 0.08)
        if math.isinf(oc):
            assert math.isinf(clr[e]) and rew[e] == 1.0
        else:
            assert abs(clr[e] - oc) <= 1e-6 + 1e-5 * oc, (e, clr[e], oc)
            assert abs(rew[e] - orw) <= 2e-5


# ------------------------------------------------------------- state pool
def test_pool_gather_scatter_roundtrip(pm):
    """scatter env states to permuted pool slots, load other states, gather
    them back: bitwise the original states (negative slots are skipped)."""
    b = scenes.clutter_batch(6, 16, (3, 12))
    sim = pm.Sim(max_envs=16, max_bodies=b.n_bodies, pool_slots=40, pool_stride=12)
    sim.set_state(b.env_offset, f32(b.state), f32(b.body))
    orig = sim.get_state()
    slots = np.arange(16, dtype=np.int32)[::-1] * 2 + 3
    sim.pool_scatter(slots)
    st2 = b.state.copy()
    st2[:, :3] += 0.5
    sim.set_state(b.env_offset, f32(st2), f32(b.body))
    moved = sim.get_state()
    gslots = slots.copy()
    gslots[5] = -1
    sim.pool_gather(gslots)
    back = sim.get_state()
    for e in range(16):
        lo, hi = b.env_offset[e], b.env_offset[e + 1]
        want = moved[lo:hi] if e == 5 else orig[lo:hi]
        assert np.array_equal(back[lo:hi], want)
    with pytest.raises(pm.PmbsError):
        sim.pool_gather(np.full(16, 40, np.int32))
