"""The allocation-free queued rollout (pmbs_sim_rollout_static, scratch in
the library's fixed device array) against the workspace-backed queued
rollout (pmbs_sim_rollout with PMBS_ROLLOUT_QUEUE): bitwise equal rewards,
counts, status and child states on consecutive calls, the second and third
smaller than the first, across the contact-class fallbacks."""
import numpy as np
import pytest

from paper_2207_06649_amd import scenes

from test_gpu_batching import Run, env_equal, grid_env, uneven_case

pytestmark = pytest.mark.gpu

SUB = 8


@pytest.fixture(scope="module")
def pm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2207_06649_amd import pmbs
    return pmbs


def static_go(r, acts, off, tgt, substeps):
    r.rew.fill_(-9.0)
    r.cnt.fill_(-9)
    r.sim.rollout_static(acts, off, tgt, n_substeps=substeps, src_slot=r.src, child_slot=r.child, max_h=5,
                         flags=0, rewards=r.rew, counts=r.cnt)
    return r.result()


def check(pm, b, acts, off, tgt, max_contacts, plan):
    ref_run = Run(pm, b, max_contacts)
    ref_run.sim.set_launch_plan(**plan)
    ref = ref_run.go(acts, off, tgt, SUB, pm.ROLLOUT_QUEUE)
    r = Run(pm, b, max_contacts)
    r.sim.set_launch_plan(**plan)
    got = static_go(r, acts, off, tgt, SUB)
    for e in range(b.n_envs):
        assert env_equal(b, e, got, ref), (max_contacts, e)
    return ref


def test_static_rollout_matches_queued_rollout(pm):
    # 1: 96 uneven envs, four of them overflowing 128 contacts (256-contact fallback)
    b, acts, off, tgt = uneven_case(5, 92, n_grid=4)
    print(f"# no-alloc call 1: {b.n_envs} envs, 256 contacts", flush=True)
    check(pm, b, acts, off, tgt, 256, dict(small_max_bodies=16))
    # 2: a smaller batch with a 30-cube grid that only the 512-contact kernel holds
    b2, acts2, off2, tgt2 = uneven_case(13, 20, n_bodies=(5, 12), region=0.3)
    b2 = scenes.concat([b2, grid_env(n=30, cols=6)])
    acts2 = np.concatenate([acts2, np.array([4, 4], np.int32)])
    off2 = np.concatenate([off2, [off2[-1] + 2]]).astype(np.int32)
    tgt2 = np.concatenate([tgt2, [0]]).astype(np.int32)
    print(f"# no-alloc call 2: {b2.n_envs} envs, 512 contacts", flush=True)
    ref2 = check(pm, b2, acts2, off2, tgt2, 512, dict(small_max_bodies=31))
    assert not (ref2[2][-1] & 1)
    # 3: smaller again, one 128-contact kernel for every env
    b3, acts3, off3, tgt3 = uneven_case(21, 12, n_bodies=(5, 15))
    print(f"# no-alloc call 3: {b3.n_envs} envs, 128 contacts", flush=True)
    check(pm, b3, acts3, off3, tgt3, 128, dict(small_max_bodies=16))
