"""Continuous-batching motion-transfer server on one GPU.

The one-GPU share of the frame-parallel pipeline (Sec. 4.7): every target
frame of a clip is transferred from the clip's first frame, so a clip's
Gaussians are uploaded once, projected and binned once (tg_preprocess,
tg_bin_sort) and stay resident while its frames arrive.  Each scheduler step
takes the ready frames of up to TG_MAX_SLOTS resident clips, up to
TG_MAX_FRAMES frames per clip, and runs them as one
tg_splat_accumulate_batch launch (one alpha/T evaluation per clip, each
frame's statistics side by side) followed by tg_solve_views and
tg_triangulate per frame.  Track uploads run on a copy stream and overlap
the compute stream; several steps may be in flight; requests that arrive
meanwhile are admitted as memory frees up.

Admission is by an HBM budget: a clip is admitted (first in, first out)
when its resident set and one frame's working set fit; a frame enters a
step when its working set fits.  Completion times come from GPU events, so
latency is arrival -> results in device memory.

`Scheduler` is the host-only policy (testable without a GPU); `Server`
executes its decisions with libtg.
"""
from __future__ import annotations

import collections
import ctypes
import time
from dataclasses import dataclass, field

from . import _lib

MAX_SLOTS = _lib.TG_MAX_SLOTS
MAX_FRAMES = _lib.TG_MAX_FRAMES


class BudgetError(RuntimeError):
    """A clip whose resident set plus one frame exceeds the whole budget."""


# ------------------------------------------------------------ byte counts
def frame_bytes(n, V, H, W):
    """Device bytes of one in-flight frame: tracks (8 B) and visibility
    (1 B) per pixel; accumulators (64 B), new 2D mean/covariance and flags
    (21 B) and the compact totals (8 B) per (view, Gaussian); output
    mean/quaternion/scale and status (44 B) per Gaussian."""
    return V * H * W * 9 + V * n * (64 + 21 + 8) + n * 44


def resident_bytes(n, V, n_cells, capacity, ws_bytes):
    """Device bytes a clip keeps while admitted: Gaussians (44 B), splat
    records, covariance, rectangle and key (64 B per (view, Gaussian)),
    depth order (4 B per (view, Gaussian)), pair list (4 B per pair), cell
    ranges (8 B per cell) and the binning workspace."""
    return n * 44 + V * n * 68 + capacity * 4 + n_cells * 8 + ws_bytes


# ------------------------------------------------------------- host policy
@dataclass
class Frame:
    clip: int
    index: int
    arrival: float
    nbytes: int
    payload: object = None
    state: str = "waiting"     # waiting -> uploading/ready -> running -> done
    credit: bool = False       # runs on its clip's reserved frame
    done: float | None = None
    result: object = None


@dataclass
class ClipState:
    cid: int
    n: int
    V: int
    H: int
    W: int
    n_frames: int
    nbytes: int
    opened: float
    state: str = "waiting"     # waiting -> admitted -> closed
    frames: list = field(default_factory=list)
    finished: int = 0
    credit_free: bool = True
    handle: object = None


class Scheduler:
    """Admission and step building under a byte budget (no device work)."""

    def __init__(self, budget_bytes, max_slots=MAX_SLOTS, max_frames=MAX_FRAMES):
        self.budget = int(budget_bytes)
        self.used = 0
        self.max_slots = max_slots
        self.max_frames = max_frames
        self.clips: dict[int, ClipState] = {}
        self.clip_queue: collections.deque[int] = collections.deque()

    # -- requests
    def open_clip(self, cid, n, V, H, W, n_frames, nbytes, now):
        if cid in self.clips:
            raise ValueError(f"clip {cid} already open")
        c = ClipState(cid, n, V, H, W, n_frames, int(nbytes), now)
        if c.nbytes + frame_bytes(n, V, H, W) > self.budget:
            raise BudgetError(f"clip {cid} needs {c.nbytes + frame_bytes(n, V, H, W)} B, budget {self.budget} B")
        self.clips[cid] = c
        self.clip_queue.append(cid)
        return c

    def arrive(self, cid, index, now, payload=None):
        c = self.clips[cid]
        f = Frame(cid, index, now, frame_bytes(c.n, c.V, c.H, c.W), payload)
        c.frames.append(f)
        return f

    # -- admission: clips first in, first out (no overtaking, so a large
    # clip is never starved by a run of small ones).  An admitted clip holds
    # its resident set plus one frame's working set, so every admitted clip
    # can always make progress.
    def admit(self):
        out = []
        while self.clip_queue:
            c = self.clips[self.clip_queue[0]]
            need = c.nbytes + frame_bytes(c.n, c.V, c.H, c.W)
            if self.used + need > self.budget:
                break
            self.clip_queue.popleft()
            self.used += need
            c.state = "admitted"
            out.append(c)
        return out

    # -- frames: bytes are reserved when a frame is taken for upload and
    # released when its step retires
    def reserve_upload(self, frame):
        """Reserve a frame's working set (the clip's own frame reserve when
        free, else the shared budget); False when neither has room."""
        c = self.clips[frame.clip]
        if c.credit_free:
            c.credit_free = False
            frame.credit = True
        elif self.used + frame.nbytes > self.budget:
            return False
        else:
            self.used += frame.nbytes
        frame.state = "uploading"
        return True

    def to_upload(self):
        """Waiting frames of admitted clips, oldest first."""
        fr = [f for c in self.clips.values() if c.state == "admitted" for f in c.frames if f.state == "waiting"]
        return sorted(fr, key=lambda f: f.arrival)

    def next_step(self, ready_clip=lambda c: True):
        """Groups [(clip, [frames])] for one launch: the clips whose oldest
        ready frame is oldest, at most max_slots clips and max_frames frames
        per clip."""
        cands = []
        for c in self.clips.values():
            if c.state != "admitted":
                continue
            fr = sorted([f for f in c.frames if f.state == "ready"], key=lambda f: f.arrival)
            if fr and ready_clip(c):
                cands.append((fr[0].arrival, c.cid, c, fr[: self.max_frames]))
        cands.sort(key=lambda x: x[:2])
        groups = [(c, fr) for _, _, c, fr in cands[: self.max_slots]]
        for _, fr in groups:
            for f in fr:
                f.state = "running"
        return groups

    def complete(self, groups):
        closed = []
        for c, frames in groups:
            for f in frames:
                f.state = "done"
                if f.credit:
                    c.credit_free = True
                else:
                    self.used -= f.nbytes
                c.finished += 1
            if c.finished == c.n_frames:
                c.state = "closed"
                self.used -= c.nbytes + frame_bytes(c.n, c.V, c.H, c.W)
                closed.append(c)
        return closed

    def idle(self):
        return all(c.state == "closed" for c in self.clips.values())


# -------------------------------------------------------------- executor
class _Resident:
    """A clip's resident device state: Gaussians, splats and bins."""

    def __init__(self, api, g, cams_host, params, capacity):
        import torch
        self.api = api
        self.g = g
        self.cams = cams_host
        self.params = params
        self.N = g.n
        self.V = len(cams_host)
        self.W = int(cams_host[0].width)
        self.H = int(cams_host[0].height)
        dev = g.means.device
        L = _lib.lib()
        self.n_cells = int(L.tg_num_cells(cams_host, self.V, self.N, ctypes.byref(params)))
        self.splats = api.SplatTensors.alloc(self.V, self.N, dev)
        self.capacity = int(capacity)
        self.bins = api.BinTensors.alloc(self.V, self.N, self.n_cells, self.capacity, dev)
        self.ws = torch.empty(api.bin_sort_ws_bytes(self.N, cams_host, params, self.capacity), dtype=torch.uint8,
                              device=dev)
        self.check = torch.zeros(2, dtype=torch.int64, pin_memory=True)
        self.event = None

    def prepare(self, stream):
        import torch
        with torch.cuda.stream(stream):
            self.api.preprocess(self.g, self.cams, self.params, self.splats)
            self.api.bin_sort(self.splats, self.N, self.cams, self.params, self.bins, self.ws)
            self.check[0].copy_(self.bins.n_pairs[0], non_blocking=True)
            self.check[1].copy_(self.bins.overflow[0].to(torch.int64), non_blocking=True)
            self.event = torch.cuda.Event()
            self.event.record(stream)

    def ready(self, stream):
        """True once binning finished without overflow; re-bins (larger
        capacity) after an overflow."""
        if self.event is None or not self.event.query():
            return False
        if int(self.check[1]) == 0:
            return True
        import torch
        self.capacity = int(int(self.check[0]) * 1.1) + 1024
        dev = self.g.means.device
        with torch.cuda.stream(stream):
            self.bins = self.api.BinTensors.alloc(self.V, self.N, self.n_cells, self.capacity, dev)
            self.ws = torch.empty(self.api.bin_sort_ws_bytes(self.N, self.cams, self.params, self.capacity),
                                  dtype=torch.uint8, device=dev)
        self.prepare(stream)
        return False


def default_capacity(n, V):
    return max(1024, 4 * n * V)


class Server:
    """Runs clips through libtg with continuous batching.

    open_clip(cid, gaussians (GaussianTensors on the device), cams, n_frames)
    submit(cid, index, disp, vis) -- host (pinned) or device tensors
    poll() -- admit, upload, launch, retire; returns finished frames
    """

    def __init__(self, budget_bytes, params=None, max_inflight=3, device="cuda", keep_intermediate=False):
        import torch
        from . import api
        self.api = api
        self.torch = torch
        self.device = torch.device(device)
        self.params = params if params is not None else _lib.default_params()
        self.sched = Scheduler(budget_bytes)
        self.compute = torch.cuda.Stream(device=self.device)
        self.copy = torch.cuda.Stream(device=self.device)
        self.max_inflight = max_inflight
        self.keep_intermediate = keep_intermediate
        self.inflight = collections.deque()     # (event, groups, buffers)
        self.pending_clips = {}
        # common origin of host and GPU clocks: the GPU reaches t0_event
        # just before the host reads t0_host
        self.t0_event = torch.cuda.Event(enable_timing=True)
        self.t0_event.record(self.compute)
        self.t0_event.synchronize()
        self.t0_host = time.perf_counter()
        self.finished = []
        self.steps = 0
        self.slots_launched = 0
        self.frames_per_step = []
        self.max_admitted = 0

    def now(self):
        return time.perf_counter() - self.t0_host

    def _gpu_time(self, ev):
        return self.t0_event.elapsed_time(ev) * 1e-3

    # -- requests
    def open_clip(self, cid, g, cams, n_frames, capacity=None, now=None):
        cams_host = cams if isinstance(cams, ctypes.Array) else _lib.cameras(cams)
        V = len(cams_host)
        W, H = int(cams_host[0].width), int(cams_host[0].height)
        cap = capacity or default_capacity(g.n, V)
        L = _lib.lib()
        ncell = int(L.tg_num_cells(cams_host, V, g.n, ctypes.byref(self.params)))
        wsb = self.api.bin_sort_ws_bytes(g.n, cams_host, self.params, cap)
        c = self.sched.open_clip(cid, g.n, V, H, W, n_frames, resident_bytes(g.n, V, ncell, cap, wsb),
                                 self.now() if now is None else now)
        self.pending_clips[cid] = (g, cams_host, cap)
        return c

    def submit(self, cid, index, disp, vis=None, now=None):
        return self.sched.arrive(cid, index, self.now() if now is None else now, payload=(disp, vis))

    # -- progress
    def _admit(self):
        for c in self.sched.admit():
            g, cams_host, cap = self.pending_clips.pop(c.cid)
            # every device buffer of the clip belongs to the compute stream
            with self.torch.cuda.stream(self.compute):
                c.handle = _Resident(self.api, g, cams_host, self.params, cap)
            c.handle.prepare(self.compute)
        n_adm = sum(1 for c in self.sched.clips.values() if c.state == "admitted")
        self.max_admitted = max(self.max_admitted, n_adm)

    def _upload(self):
        torch = self.torch
        for f in self.sched.to_upload():
            if not self.sched.reserve_upload(f):
                return
            disp, vis = f.payload
            with torch.cuda.stream(self.copy):
                d = torch.empty(disp.shape, dtype=torch.float32, device=self.device)
                d.copy_(disp, non_blocking=True)
                v = None
                if vis is not None:
                    v = torch.empty(vis.shape, dtype=torch.uint8, device=self.device)
                    v.copy_(vis, non_blocking=True)
                ev = torch.cuda.Event()
                ev.record(self.copy)
            # the buffers are read on the compute stream too
            d.record_stream(self.compute)
            if v is not None:
                v.record_stream(self.compute)
            f.payload = (d, v, ev)
            f.state = "ready"

    def _launch(self):
        torch = self.torch
        if len(self.inflight) >= self.max_inflight:
            return False
        groups = self.sched.next_step(ready_clip=lambda c: c.handle.ready(self.compute))
        if not groups:
            return False
        api = self.api
        slots = []
        with torch.cuda.stream(self.compute):
            for c, frames in groups:
                r = c.handle
                for f in frames:
                    self.compute.wait_event(f.payload[2])
                accs = [torch.zeros(r.V, r.N, 16, dtype=torch.float32, device=self.device) for _ in frames]
                slots.append(dict(splats=r.splats, bins=r.bins, n=r.N, cams=r.cams,
                                  disp=[f.payload[0] for f in frames], vis=[f.payload[1] for f in frames],
                                  acc=accs))
            api.splat_accumulate_batch(slots, self.params)
            for (c, frames), sl in zip(groups, slots):
                r = c.handle
                VN = (r.V, r.N)
                for f, acc in zip(frames, sl["acc"]):
                    mu = torch.empty(*VN, 2, dtype=torch.float32, device=self.device)
                    cov = torch.empty(*VN, 3, dtype=torch.float32, device=self.device)
                    vfl = torch.empty(*VN, dtype=torch.uint8, device=self.device)
                    wn = torch.empty(*VN, 2, dtype=torch.float32, device=self.device)
                    st = torch.empty(r.N, dtype=torch.int32, device=self.device)
                    g = r.g
                    out = api.GaussianTensors(torch.empty_like(g.means), torch.empty_like(g.quats),
                                              torch.empty_like(g.scales), g.opacity, g.sh, g.sh_degree,
                                              g.scale_mode, g.opacity_mode)
                    api.solve_views(acc, r.splats, r.N, r.V, self.params, mu, cov, vfl, wn)
                    api.triangulate(mu, cov, vfl, wn, r.splats, g, r.cams, self.params, out, st)
                    f.result = (out, st, acc, mu, cov, vfl) if self.keep_intermediate else (out, st)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(self.compute)
        # the step holds its buffers until it retires
        self.inflight.append((ev, groups, slots))
        for c, frames in groups:
            for f in frames:
                f.payload = None
        self.steps += 1
        self.slots_launched += len(groups)
        self.frames_per_step.append(sum(len(fr) for _, fr in groups))
        return True

    def _retire(self):
        done = []
        while self.inflight and self.inflight[0][0].query():
            ev, groups, _ = self.inflight.popleft()
            t = self._gpu_time(ev)
            for c, frames in groups:
                for f in frames:
                    f.done = t
                    done.append(f)
            for c in self.sched.complete(groups):
                c.handle = None      # the clip's resident set is released
        self.finished += done
        return done

    def poll(self):
        self._retire()
        self._admit()
        self._upload()
        while self._launch():
            pass
        return self._retire()

    def drain(self, sleep=0.0002):
        """Process until every opened clip has finished (all of its frames
        must have been submitted)."""
        while not self.sched.idle() or self.inflight:
            self.poll()
            if self.inflight:
                time.sleep(sleep)
