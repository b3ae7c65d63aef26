"""Host policy of libtg's continuous-batching server (tg_serve_*) in dry mode
(no GPU: the arena is an address range that is never touched, steps end
when the test says so): admission by the arena budget, first in first out
without overtaking, step composition (oldest ready frame first, entries of
at most TG_MAX_FRAMES frames, at most max_slots entries, max_frames frames
of a clip per step), the budget never exceeded, every frame finished once,
everything released at the end."""
from types import SimpleNamespace

import numpy as np
import pytest

import synth
from paper_2604_02586_amd import _lib
from paper_2604_02586_amd.serving import BudgetError, Server, stream_bytes


def _clip(n=1000, V=2, W=64, H=48):
    return SimpleNamespace(n=n), synth.ring_cameras(V, 3.0, W, H)


def _need(n=1000, V=2, W=64, H=48):
    g, cams = _clip(n, V, W, H)
    r, fh, _ = stream_bytes(cams, n)
    return r + fh


def _finish(srv, k=1000, t=1.0):
    _lib.lib().tg_serve_dry_complete(srv.h, k, t)
    return srv.poll()


def test_budget_rejects_a_clip_that_can_never_fit():
    srv = Server(budget_bytes=_need() - 1, dry=True)
    with pytest.raises(BudgetError):
        srv.open_clip(*_clip())
    srv2 = Server(budget_bytes=_need(), dry=True)
    srv2.open_clip(*_clip())


def test_fifo_admission_without_overtaking():
    a, b, c = _need(n=20000), _need(n=15000), _need(n=1000)
    assert c + 4096 < b < a
    srv = Server(budget_bytes=a + c + 4096, dry=True)
    sa = srv.open_clip(*_clip(n=20000), arrival=0.0)
    sb = srv.open_clip(*_clip(n=15000), arrival=0.1)   # does not fit beside a
    sc = srv.open_clip(*_clip(n=1000), arrival=0.2)    # would fit, must wait for b
    srv.step()
    st = srv.stats()
    assert st["admitted_streams"] == 1 and st["waiting_streams"] == 2
    # a's resident set and frame reserve (its binning workspace is already
    # released: dry binning completes at once)
    assert 0 < st["arena_used"] <= a
    srv.submit(sa, 0, None, arrival=0.3)
    assert srv.step() == 1
    done = _finish(srv)
    assert [(f.stream, f.index, f.step) for f in done] == [(sa, 0, 0)]
    srv.close(sa)
    srv.step()
    st = srv.stats()
    # a released: b and then c admitted (both fit once a is gone)
    assert st["admitted_streams"] == 2 and st["waiting_streams"] == 0
    assert st["arena_used"] <= a + c + 4096
    for s in (sb, sc):
        srv.close(s)
    srv.step()
    assert srv.stats()["arena_used"] == 0 and srv.stats()["waiting_streams"] == 0


def test_step_composition_limits_and_order():
    srv = Server(budget_bytes=1 << 40, max_slots=3, max_frames=2, dry=True)
    ids = [srv.open_clip(*_clip(), arrival=float(k)) for k in range(5)]
    t = 10.0
    for k in range(3):
        for i in (4, 3, 2, 1, 0):
            t += 1.0
            srv.submit(ids[i], k, None, arrival=t)
    assert srv.step() >= 1
    done = _finish(srv, k=1)
    first = sorted([f for f in done if f.step == 0], key=lambda f: (f.entry, f.arrival))
    # three clips whose oldest ready frame is oldest: 4, 3, 2; two frames each
    entries = {}
    for f in first:
        entries.setdefault(f.entry, []).append(f)
    assert [entries[e][0].stream for e in sorted(entries)] == [ids[4], ids[3], ids[2]]
    assert all(len(v) == 2 for v in entries.values())
    assert all(v[0].arrival < v[1].arrival for v in entries.values())
    assert all(v[0].index == 0 and v[1].index == 1 for v in entries.values())


def test_eight_frames_of_one_clip_form_two_entries():
    srv = Server(budget_bytes=1 << 40, max_slots=8, max_frames=8, dry=True)
    s = srv.open_clip(*_clip(), arrival=0.0)
    for k in range(9):
        srv.submit(s, k, None, arrival=1.0 + k)
    srv.step()
    done = _finish(srv, k=1)
    first = [f for f in done if f.step == 0]
    assert sorted(f.index for f in first) == list(range(8))
    assert sorted(set(f.entry for f in first)) == [0, 1]
    assert all(sum(1 for f in first if f.entry == e) == _lib.TG_MAX_FRAMES for e in (0, 1))


def test_randomised_run_respects_budget_and_finishes_every_frame():
    rng = np.random.default_rng(0)
    specs = []
    for _ in range(14):
        specs.append(dict(n=int(rng.integers(1000, 40000)), V=int(rng.integers(2, 7)),
                          W=int(rng.choice([64, 96, 160])), H=int(rng.choice([48, 64, 120])),
                          frames=int(rng.integers(1, 9))))
    budget = max(_need(s["n"], s["V"], s["W"], s["H"]) for s in specs) * 3
    srv = Server(budget_bytes=budget, max_slots=4, max_frames=8, max_inflight=3, dry=True)
    sids = []
    for k, s in enumerate(specs):
        sids.append(srv.open_clip(*_clip(s["n"], s["V"], s["W"], s["H"]), arrival=k * 0.01))
    pending = [(ci, f) for ci, s in enumerate(specs) for f in range(s["frames"])]
    rng.shuffle(pending)
    nxt = [0] * len(specs)
    t, got, peak = 1.0, [], 0
    total = sum(s["frames"] for s in specs)
    for _ in range(100000):
        if len(got) == total:
            break
        # a few arrivals, in each clip's own order
        for _ in range(int(rng.integers(0, 3))):
            cands = [p for p in pending if nxt[p[0]] == p[1]]
            if not cands:
                break
            ci, f = cands[0]
            pending.remove((ci, f))
            t += 0.01
            srv.submit(sids[ci], f, None, arrival=t)
            nxt[ci] += 1
            if nxt[ci] == specs[ci]["frames"]:
                srv.close(sids[ci])
        srv.step()
        st = srv.stats()
        peak = max(peak, st["arena_used"])
        assert st["arena_used"] <= budget
        assert st["inflight_steps"] <= 3
        if st["inflight_steps"] and rng.random() < 0.6:
            _lib.lib().tg_serve_dry_complete(srv.h, int(rng.integers(1, 3)), t)
        got += srv.collect()
    keys = [(f.stream, f.index) for f in got]
    assert len(keys) == len(set(keys)) == sum(s["frames"] for s in specs)
    # each clip's frames finish in submission order
    for sid in sids:
        idx = [f.index for f in got if f.stream == sid]
        assert idx == sorted(idx)
    srv.step()
    st = srv.stats()
    assert st["arena_used"] == 0 and st["admitted_streams"] == 0 and st["waiting_streams"] == 0
    assert st["steps"] < len(keys)          # batching happened
    assert peak <= budget and st["arena_peak"] == peak


def test_closing_a_waiting_clip_withdraws_it():
    srv = Server(budget_bytes=_need() + 1000, dry=True)
    a = srv.open_clip(*_clip())
    b = srv.open_clip(*_clip())
    srv.step()
    assert srv.stats()["waiting_streams"] == 1
    srv.close(b)
    assert srv.stats()["waiting_streams"] == 0
    srv.close(a)
    srv.step()
    assert srv.stats()["arena_used"] == 0


def test_invalid_requests():
    srv = Server(budget_bytes=1 << 30, dry=True)
    with pytest.raises(_lib.TGError):
        srv.submit(12345, 0, None)            # unknown stream
    s = srv.open_clip(*_clip())
    srv.close(s)
    with pytest.raises(_lib.TGError):
        srv.submit(s, 0, None)                # closed stream
    with pytest.raises(_lib.TGError):
        Server(budget_bytes=1 << 30, max_slots=_lib.TG_MAX_SLOTS + 1, dry=True)
