"""Driver of libtg's continuous-batching motion-transfer server (tg_serve_*).

The server itself -- admission of clips (streams) by an HBM budget, first
in first out, resident splats and bins per clip, track uploads on a copy
stream, steps of one batched accumulate and one fused update launch, latency
from GPU events -- is host C++ inside libtg (Sec. 4.7: every target frame of
a clip is transferred from the clip's first frame).  This module only owns
the buffers the server needs (the device arena that is the budget, pinned
host scratch, two HIP streams, the output tensors of each frame) and
marshals calls.
"""
from __future__ import annotations

import ctypes
import time
from dataclasses import dataclass, field

from . import _lib

MAX_SLOTS = _lib.TG_MAX_SLOTS
MAX_FRAMES = _lib.TG_MAX_FRAMES
TG_ERR_BUDGET = 6


class BudgetError(RuntimeError):
    """A clip whose resident set plus one frame exceeds the whole budget."""


def stream_bytes(cams, n, params=None):
    """(resident, frame with host tracks, frame with device tracks) bytes a
    clip needs in the server's arena (tg_serve_stream_bytes)."""
    cams = cams if isinstance(cams, ctypes.Array) else _lib.cameras(cams)
    params = params if params is not None else _lib.default_params()
    r, fh, fd = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _lib.check("tg_serve_stream_bytes", _lib.lib().tg_serve_stream_bytes(
        cams, len(cams), int(n), ctypes.byref(params), ctypes.byref(r), ctypes.byref(fh), ctypes.byref(fd)))
    return r.value, fh.value, fd.value


@dataclass
class Frame:
    """A submitted frame; `result` is (GaussianTensors, status) once done."""
    stream: int
    index: int
    arrival: float
    result: object = None
    done: float | None = None
    step: int = -1
    entry: int = -1
    status: int = 0
    keep: list = field(default_factory=list)


class Server:
    """open_clip(g, cams) -> stream id; submit(sid, index, disp, vis);
    close(sid); poll() -> finished frames; drain()."""

    def __init__(self, budget_bytes, params=None, max_inflight=3, max_frames=2 * MAX_FRAMES, max_slots=MAX_SLOTS,
                 device="cuda", dry=False):
        self.params = params if params is not None else _lib.default_params()
        self.dry = bool(dry)
        L = _lib.lib()
        cfg = _lib.ServeConfig()
        cfg.arena_bytes = int(budget_bytes)
        cfg.max_inflight = int(max_inflight)
        cfg.max_frames = int(max_frames)
        cfg.max_slots = int(max_slots)
        cfg.dry = 1 if self.dry else 0
        if not self.dry:
            import torch
            self.torch = torch
            self.device = torch.device(device)
            self.arena = torch.empty(int(budget_bytes), dtype=torch.uint8, device=self.device)
            self.host_scratch = torch.zeros(_lib.TG_SERVE_HOST_BYTES, dtype=torch.uint8).pin_memory()
            self.compute = torch.cuda.Stream(device=self.device)
            self.copy = torch.cuda.Stream(device=self.device)
            cfg.arena = self.arena.data_ptr()
            cfg.host_scratch = self.host_scratch.data_ptr()
            cfg.compute_stream = self.compute.cuda_stream
            cfg.copy_stream = self.copy.cuda_stream
        h = ctypes.c_void_p()
        _lib.check("tg_serve_create", L.tg_serve_create(ctypes.byref(cfg), ctypes.byref(self.params), ctypes.byref(h)))
        self.h = h
        self.clips = {}        # stream id -> (GaussianTensors, cams)
        self.frames = {}       # (stream id, index) -> Frame
        self.finished = []
        self._done_buf = (_lib.ServeDone * 256)()

    # -- clock
    def now(self):
        return _lib.lib().tg_serve_now(self.h)

    # -- requests
    def open_clip(self, g, cams, arrival=None):
        cams = cams if isinstance(cams, ctypes.Array) else _lib.cameras(cams)
        sid = ctypes.c_int64()
        gc = g.c() if not self.dry else _lib.Gaussians()
        if not self.dry:
            # the Gaussians were written on the caller's stream
            self.compute.wait_stream(self.torch.cuda.current_stream())
        code = _lib.lib().tg_serve_open_stream(self.h, ctypes.byref(gc), int(g.n), cams, len(cams),
                                               self.now() if arrival is None else float(arrival), ctypes.byref(sid))
        if code == TG_ERR_BUDGET:
            raise BudgetError(f"clip of {g.n} Gaussians x {len(cams)} views does not fit the budget")
        _lib.check("tg_serve_open_stream", code)
        self.clips[sid.value] = (g, cams)
        return sid.value

    def submit(self, sid, index, disp, vis=None, arrival=None):
        """disp [V,H,W,2] float32 and vis [V,H,W] uint8 (or None), both on the
        host (pinned) or both on the device."""
        arrival = self.now() if arrival is None else float(arrival)
        fr = Frame(sid, index, arrival)
        if self.dry:
            go = _lib.Gaussians()
            _lib.check("tg_serve_submit", _lib.lib().tg_serve_submit(self.h, sid, index, None, None, 1,
                                                                     ctypes.byref(go), None, arrival))
            self.frames[sid, index] = fr
            return fr
        torch = self.torch
        from . import api
        g, _ = self.clips[sid]
        host = not disp.is_cuda
        if host and not disp.is_pinned():
            disp = disp.pin_memory()
        if vis is not None and host and not vis.is_pinned():
            vis = vis.pin_memory()
        if not host:
            self.compute.wait_stream(torch.cuda.current_stream())
        out = api.GaussianTensors(torch.empty_like(g.means), torch.empty_like(g.quats), torch.empty_like(g.scales),
                                  g.opacity, g.sh, g.sh_degree, g.scale_mode, g.opacity_mode)
        st = torch.empty(g.n, dtype=torch.int32, device=self.device)
        go = out.c()
        fr.keep = [disp, vis, go]
        fr.result = (out, st)
        _lib.check("tg_serve_submit", _lib.lib().tg_serve_submit(
            self.h, sid, index, disp.data_ptr(), None if vis is None else vis.data_ptr(), 1 if host else 0,
            ctypes.byref(go), st.data_ptr(), arrival))
        self.frames[sid, index] = fr
        return fr

    def close(self, sid):
        _lib.check("tg_serve_close_stream", _lib.lib().tg_serve_close_stream(self.h, sid))

    # -- progress
    def step(self):
        n = ctypes.c_int32()
        _lib.check("tg_serve_step", _lib.lib().tg_serve_step(self.h, ctypes.byref(n)))
        return n.value

    def collect(self):
        """Finished frames since the last call (their outputs are complete)."""
        out = []
        n = ctypes.c_int32()
        while True:
            _lib.check("tg_serve_poll", _lib.lib().tg_serve_poll(self.h, self._done_buf, len(self._done_buf),
                                                                 ctypes.byref(n)))
            for i in range(n.value):
                d = self._done_buf[i]
                fr = self.frames.pop((d.stream_id, d.frame_id))
                fr.done, fr.step, fr.entry, fr.status = d.done, d.step, d.entry, d.status
                fr.keep = []
                out.append(fr)
            if n.value < len(self._done_buf):
                break
        for fr in out:
            if fr.status:
                raise _lib.TGError(f"frame {fr.index} of stream {fr.stream}", fr.status)
        self.finished += out
        return out

    def poll(self):
        self.step()
        return self.collect()

    def stats(self):
        st = _lib.ServeStats()
        _lib.check("tg_serve_get_stats", _lib.lib().tg_serve_get_stats(self.h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in st._fields_}

    def busy(self):
        s = self.stats()
        return bool(self.frames) or s["inflight_steps"] > 0

    def drain(self, sleep=0.0002):
        """Process until every submitted frame is done."""
        while self.frames:
            self.poll()
            if self.frames:
                time.sleep(sleep)

    def destroy(self):
        if getattr(self, "h", None):
            _lib.check("tg_serve_destroy", _lib.lib().tg_serve_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
