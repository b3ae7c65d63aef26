"""Host-side policy of the continuous-batching server (no GPU): admission by
byte budget, first-in-first-out clips, step composition, accounting."""
import numpy as np
import pytest

from paper_2604_02586_amd.serving import BudgetError, Scheduler, frame_bytes


def _open(s, cid, n=1000, V=2, H=16, W=16, frames=2, nbytes=1000, now=0.0):
    return s.open_clip(cid, n, V, H, W, frames, nbytes, now)


def test_budget_rejects_a_clip_that_can_never_fit():
    s = Scheduler(budget_bytes=10_000)
    with pytest.raises(BudgetError):
        _open(s, 0, n=1000, nbytes=5000)   # one frame alone is ~175 kB


def test_fifo_admission_under_budget():
    fb = frame_bytes(1000, 2, 16, 16)
    s = Scheduler(budget_bytes=3 * (10_000 + fb) + fb - 1)
    _open(s, 0, nbytes=2 * (10_000 + fb), frames=1)   # large
    _open(s, 1, nbytes=10_000, frames=1)
    _open(s, 2, nbytes=10_000, frames=1)
    got = [c.cid for c in s.admit()]
    assert got == [0]                  # 1 misses by one byte
    assert s.used == 2 * (10_000 + fb) + fb
    f0 = s.arrive(0, 1, now=0.1)
    assert s.reserve_upload(f0)
    f0.state = "ready"
    g = s.next_step()
    assert [(c.cid, [f.index for f in fr]) for c, fr in g] == [(0, [1])]
    s.complete(g)
    assert s.clips[0].state == "closed" and s.used == 0
    assert [c.cid for c in s.admit()] == [1, 2]


def test_no_overtaking_of_a_waiting_clip():
    fb = frame_bytes(1000, 2, 16, 16)
    s = Scheduler(budget_bytes=2 * (10_000 + fb))
    _open(s, 0, nbytes=10_000)
    _open(s, 1, nbytes=10_000 + 1)        # does not fit beside clip 0
    _open(s, 2, nbytes=100)               # would fit, but must wait for 1
    assert [c.cid for c in s.admit()] == [0]
    assert s.admit() == []


def test_step_composition_limits_and_order():
    s = Scheduler(budget_bytes=1 << 40, max_slots=3, max_frames=2)
    for cid in range(5):
        _open(s, cid, frames=5, now=cid)
    s.admit()
    t = 0.0
    for k in range(3):
        for cid in (4, 3, 2, 1, 0):
            t += 1.0
            f = s.arrive(cid, k + 1, now=t)
            assert s.reserve_upload(f)
            f.state = "ready"
    g = s.next_step()
    # three clips whose oldest ready frame is oldest: 4, 3, 2; two frames each
    assert [c.cid for c, _ in g] == [4, 3, 2]
    assert all(len(fr) == 2 for _, fr in g)
    assert all(fr[0].arrival < fr[1].arrival for _, fr in g)
    assert all(f.state == "running" for _, fr in g for f in fr)


def test_simulated_run_respects_budget_and_finishes_every_frame():
    rng = np.random.default_rng(0)
    budget = 40_000_000
    s = Scheduler(budget_bytes=budget, max_slots=4, max_frames=3)
    clips, t = [], 0.0
    for cid in range(12):
        n = int(rng.integers(1000, 50_000))
        V = int(rng.integers(2, 6))
        frames = int(rng.integers(1, 6))
        _open(s, cid, n=n, V=V, H=64, W=64, frames=frames, nbytes=n * V * 70, now=t)
        clips.append((cid, frames))
    pending = [(cid, k) for cid, fr in clips for k in range(1, fr + 1)]
    rng.shuffle(pending)
    order = {cid: 0 for cid, _ in clips}
    inflight, done, steps = [], 0, 0
    while not s.idle():
        s.admit()
        # frames of admitted clips arrive in order
        for i, (cid, k) in enumerate(list(pending)):
            if s.clips[cid].state == "admitted" and order[cid] == k - 1:
                t += 0.01
                s.arrive(cid, k, now=t)
                order[cid] = k
                pending.remove((cid, k))
                break
        for f in s.to_upload():
            if not s.reserve_upload(f):
                break
            f.state = "ready"
        assert s.used <= budget
        g = s.next_step()
        if g:
            inflight.append(g)
            steps += 1
        if inflight and (len(inflight) > 2 or not g):
            done_g = inflight.pop(0)
            s.complete(done_g)
            done += sum(len(fr) for _, fr in done_g)
    assert done == sum(fr for _, fr in clips)
    assert s.used == 0 and steps >= 1
