"""Python API over libtg.  Torch provides device memory and streams only;
every step of the method runs in the HIP kernels behind the C ABI.

The thin wrappers (`preprocess`, `bin_sort`, `splat_accumulate`,
`solve_views`, `triangulate`, `bin_expand`) mirror the C entry points of
include/tg.h one to one.  `MotionTransfer` owns the buffers of one scene
shape (N Gaussians, V views of one resolution) and runs a frame.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import check, lib

__all__ = ["GaussianTensors", "SplatTensors", "BinTensors", "MotionTransfer", "preprocess", "bin_sort", "bin_sort_static",
           "splat_accumulate", "splat_accumulate_batch", "regularize", "solve_views", "triangulate", "solve_triangulate",
           "solve_triangulate_batch", "cameras_device", "bin_expand", "stream_ptr", "default_params"]

default_params = _lib.default_params


def stream_ptr(stream=None) -> ctypes.c_void_p:
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("libtg takes device tensors only")
    if not t.is_contiguous():
        raise ValueError("libtg takes contiguous tensors only")
    return ctypes.c_void_p(t.data_ptr())


@dataclass
class GaussianTensors:
    means: torch.Tensor          # [N,3] f32
    quats: torch.Tensor          # [N,4] f32 (w,x,y,z)
    scales: torch.Tensor         # [N,3] f32 (linear or log)
    opacity: torch.Tensor        # [N] f32 (activated or logit)
    sh: torch.Tensor | None = None   # [N,K,3] f32
    sh_degree: int = 0
    scale_mode: int = 0
    opacity_mode: int = 0

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def c(self) -> _lib.Gaussians:
        return _lib.Gaussians(_ptr(self.means), _ptr(self.quats), _ptr(self.scales), _ptr(self.opacity),
                              _ptr(self.sh), int(self.sh_degree), int(self.scale_mode), int(self.opacity_mode), 0)

    @staticmethod
    def from_scene(scene, device="cuda", sh=False):
        t = lambda a: torch.as_tensor(a, dtype=torch.float32).to(device).contiguous()
        g = GaussianTensors(t(scene.means), t(scene.quats), t(scene.scales), t(scene.opacity))
        if sh and scene.sh is not None:
            k = scene.sh.shape[1] // 3
            g.sh = t(scene.sh).reshape(-1, k, 3).contiguous()
            g.sh_degree = int(round(k ** 0.5)) - 1
        return g

    def clone(self):
        return GaussianTensors(self.means.clone(), self.quats.clone(), self.scales.clone(), self.opacity.clone(),
                               None if self.sh is None else self.sh.clone(), self.sh_degree, self.scale_mode,
                               self.opacity_mode)


@dataclass
class SplatTensors:
    rec: torch.Tensor       # [V,N,8] f32
    cov2d: torch.Tensor     # [V,N,3] f32
    rect: torch.Tensor      # [V,N,4] int16 storage of uint16
    key: torch.Tensor       # [V,N] int32 storage of uint32
    colors: torch.Tensor | None = None
    clamped: torch.Tensor | None = None

    @staticmethod
    def alloc(V, N, device="cuda", colors=False):
        z = lambda *s, dt=torch.float32: torch.empty(*s, dtype=dt, device=device)
        return SplatTensors(z(V, N, 8), z(V, N, 3), z(V, N, 4, dt=torch.int16), z(V, N, dt=torch.int32),
                            z(V, N, 3) if colors else None, z(V, N, 3, dt=torch.uint8) if colors else None)

    def c(self) -> _lib.Splats:
        return _lib.Splats(_ptr(self.rec), _ptr(self.cov2d), _ptr(self.rect), _ptr(self.key), _ptr(self.colors),
                           _ptr(self.clamped))


@dataclass
class BinTensors:
    order: torch.Tensor        # [V,N] int32 (uint32 ids)
    cell_ids: torch.Tensor     # [capacity] int32
    cell_ranges: torch.Tensor  # [n_cells,2] int32
    n_pairs: torch.Tensor      # [1] int64
    overflow: torch.Tensor     # [1] int32
    capacity: int

    @staticmethod
    def alloc(V, N, n_cells, capacity, device="cuda"):
        return BinTensors(torch.empty(V, N, dtype=torch.int32, device=device),
                          torch.empty(max(capacity, 1), dtype=torch.int32, device=device),
                          torch.empty(n_cells, 2, dtype=torch.int32, device=device),
                          torch.zeros(1, dtype=torch.int64, device=device),
                          torch.zeros(1, dtype=torch.int32, device=device), int(capacity))

    def c(self) -> _lib.Bins:
        return _lib.Bins(_ptr(self.order), _ptr(self.cell_ids), _ptr(self.cell_ranges), _ptr(self.n_pairs),
                         _ptr(self.overflow), int(self.capacity))


# ---------------------------------------------------------------- wrappers
def preprocess(g: GaussianTensors, cams, params, out: SplatTensors, stream=None):
    cams = cams if isinstance(cams, ctypes.Array) else _lib.cameras(cams)
    gc, oc = g.c(), out.c()
    check("tg_preprocess", lib().tg_preprocess(ctypes.byref(gc), g.n, cams, len(cams), ctypes.byref(params),
                                               ctypes.byref(oc), stream_ptr(stream)))


def acc_zero(acc: torch.Tensor, stream=None):
    """tg_acc_zero over every record of `acc` ([..., 16] float32)."""
    if acc.dtype != torch.float32 or acc.numel() % 16:
        raise ValueError("acc must be float32 records of 16")
    check("tg_acc_zero", lib().tg_acc_zero(_ptr(acc), acc.numel() // 16, stream_ptr(stream)))


def bin_sort_ws_bytes(n, cams, params, capacity) -> int:
    cams = cams if isinstance(cams, ctypes.Array) else _lib.cameras(cams)
    sc = _lib.Splats()
    b = _lib.Bins()
    b.capacity = int(capacity)
    nb = ctypes.c_size_t(0)
    check("tg_bin_sort", lib().tg_bin_sort(ctypes.byref(sc), n, cams, len(cams), ctypes.byref(params),
                                           ctypes.byref(b), None, ctypes.byref(nb), None))
    return int(nb.value)


def bin_sort(s: SplatTensors, n, cams, params, bins: BinTensors, ws: torch.Tensor, stream=None):
    cams = cams if isinstance(cams, ctypes.Array) else _lib.cameras(cams)
    sc, bc = s.c(), bins.c()
    nb = ctypes.c_size_t(ws.numel() * ws.element_size())
    check("tg_bin_sort", lib().tg_bin_sort(ctypes.byref(sc), n, cams, len(cams), ctypes.byref(params),
                                           ctypes.byref(bc), _ptr(ws), ctypes.byref(nb), stream_ptr(stream)))


def bin_sort_static(s: SplatTensors, n, cams, params, bins: BinTensors, stream=None):
    """tg_bin_sort_static: the binning with the library's own scratch (no
    workspace argument, nothing allocated)."""
    cams = cams if isinstance(cams, ctypes.Array) else _lib.cameras(cams)
    sc, bc = s.c(), bins.c()
    check("tg_bin_sort_static", lib().tg_bin_sort_static(ctypes.byref(sc), n, cams, len(cams), ctypes.byref(params),
                                                         ctypes.byref(bc), stream_ptr(stream)))


def splat_accumulate(s: SplatTensors, bins: BinTensors, n, cams, disp, vis, params, acc, t_final=None,
                     stats=None, stream=None):
    cams = cams if isinstance(cams, ctypes.Array) else _lib.cameras(cams)
    sc, bc = s.c(), bins.c()
    check("tg_splat_accumulate", lib().tg_splat_accumulate(
        ctypes.byref(sc), ctypes.byref(bc), n, cams, len(cams), _ptr(disp), _ptr(vis), ctypes.byref(params),
        _ptr(acc), _ptr(t_final), _ptr(stats), stream_ptr(stream)))


def _addr(t):
    p = _ptr(t)
    return None if p is None else p.value


def splat_accumulate_batch(slots, params, stats=None, stream=None):
    """One launch over several Gaussian sets, each with F <= TG_MAX_FRAMES
    frames of tracks sharing its alpha T.  slots: sequence of dicts with keys
    splats, bins, n, cams, disp, vis, acc, t_final (optional); disp / vis /
    acc are per-frame sequences (or tensors whose leading axis is the frame)
    of [V,H,W,2] / [V,H,W] uint8 or None / [V,N,16] zeroed."""
    if len(slots) > _lib.TG_MAX_SLOTS:
        raise ValueError(f"at most {_lib.TG_MAX_SLOTS} slots per launch")
    keep = []
    arr = (_lib.AccSlot * max(1, len(slots)))()
    for i, sl in enumerate(slots):
        cams = sl["cams"] if isinstance(sl["cams"], ctypes.Array) else _lib.cameras(sl["cams"])
        sc, bc = sl["splats"].c(), sl["bins"].c()
        keep += [cams, sc, bc]
        disp = list(sl["disp"])
        acc = list(sl["acc"])
        vis = sl.get("vis")
        vis = [None] * len(disp) if vis is None else list(vis)
        if not (len(disp) == len(acc) == len(vis)) or not 1 <= len(disp) <= _lib.TG_MAX_FRAMES:
            raise ValueError("disp, vis and acc need one entry per frame, 1..TG_MAX_FRAMES frames")
        arr[i].s = ctypes.addressof(sc)
        arr[i].bins = ctypes.addressof(bc)
        arr[i].cams = ctypes.addressof(cams)
        arr[i].N = int(sl["n"])
        arr[i].V = len(cams)
        arr[i].F = len(disp)
        for f in range(len(disp)):
            arr[i].disp[f] = _addr(disp[f])
            arr[i].vis[f] = _addr(vis[f])
            arr[i].acc[f] = _addr(acc[f])
        arr[i].t_final = _addr(sl.get("t_final"))
    check("tg_splat_accumulate_batch", lib().tg_splat_accumulate_batch(
        arr, len(slots), ctypes.byref(params), _ptr(stats), stream_ptr(stream)))
    del keep


def regularize_ws_bytes(n) -> int:
    nb = ctypes.c_size_t(0)
    check("tg_regularize", lib().tg_regularize(None, None, None, None, int(n), 1, ctypes.byref(_lib.default_params()),
                                               None, ctypes.byref(nb), None, None, None))
    return int(nb.value)


def regularize(g_ref: GaussianTensors, g_upd: GaussianTensors, status, acc, params, g_out: GaussianTensors,
               reg_status, ws=None, stream=None):
    """Motion regularisation (tg_regularize); acc [V,N,16]."""
    n = g_ref.n
    if ws is None:
        ws = torch.empty(regularize_ws_bytes(n), dtype=torch.uint8, device=g_ref.means.device)
    nb = ctypes.c_size_t(ws.numel())
    gr, gu, go = g_ref.c(), g_upd.c(), g_out.c()
    check("tg_regularize", lib().tg_regularize(ctypes.byref(gr), ctypes.byref(gu), _ptr(status), _ptr(acc), n,
                                               int(acc.shape[0]), ctypes.byref(params), _ptr(ws), ctypes.byref(nb),
                                               ctypes.byref(go), _ptr(reg_status), stream_ptr(stream)))


def solve_views(acc, s: SplatTensors, n, V, params, mu_new, cov_new, vflags, wn=None, stream=None):
    """wn: optional [V,N,2] float32 output of the compact totals (alpha, pixels)."""
    sc = s.c()
    check("tg_solve_views", lib().tg_solve_views(_ptr(acc), ctypes.byref(sc), n, V, ctypes.byref(params),
                                                 _ptr(mu_new), _ptr(cov_new), _ptr(vflags),
                                                 _ptr(wn) if wn is not None else None, stream_ptr(stream)))


def triangulate(mu_new, cov_new, vflags, wn, s: SplatTensors, g_in: GaussianTensors, cams, params,
                g_out: GaussianTensors, status, stream=None):
    """wn: [V,N,2] totals written by solve_views."""
    cams = cams if isinstance(cams, ctypes.Array) else _lib.cameras(cams)
    sc, gi, go = s.c(), g_in.c(), g_out.c()
    check("tg_triangulate", lib().tg_triangulate(
        _ptr(mu_new), _ptr(cov_new), _ptr(vflags), _ptr(wn), ctypes.byref(sc), ctypes.byref(gi), g_in.n, cams,
        len(cams), ctypes.byref(params), ctypes.byref(go), _ptr(status), stream_ptr(stream)))


def solve_triangulate(acc, s: SplatTensors, g_in: GaussianTensors, cams, params, g_out: GaussianTensors, status,
                      stream=None):
    """tg_solve_triangulate: per-view solves and the multi-view update in one
    launch, nothing stored in between."""
    cams = cams if isinstance(cams, ctypes.Array) else _lib.cameras(cams)
    sc, gi, go = s.c(), g_in.c(), g_out.c()
    check("tg_solve_triangulate", lib().tg_solve_triangulate(
        _ptr(acc), ctypes.byref(sc), ctypes.byref(gi), g_in.n, cams, len(cams), ctypes.byref(params),
        ctypes.byref(go), _ptr(status), stream_ptr(stream)))


def cameras_device(cams, device) -> torch.Tensor:
    """The cameras as a device array ([V,20] float32, the tg_camera layout)
    for tg_solve_triangulate_batch."""
    cams = cams if isinstance(cams, ctypes.Array) else _lib.cameras(cams)
    import numpy as np
    host = np.frombuffer(bytes(cams), dtype=np.float32).reshape(len(cams), -1).copy()
    return torch.from_numpy(host).to(device)


def solve_triangulate_batch(slots, params, stream=None):
    """One fused update launch over several Gaussian sets and frames.
    slots: sequence of dicts with keys splats, g_in (GaussianTensors), cams
    (device tensor from cameras_device), n, V, acc (per-frame [V,N,16]),
    g_out (per-frame GaussianTensors), status (per-frame [N] int32 or None)."""
    if len(slots) > _lib.TG_MAX_SLOTS:
        raise ValueError(f"at most {_lib.TG_MAX_SLOTS} slots per launch")
    keep = []
    arr = (_lib.UpdSlot * max(1, len(slots)))()
    for i, sl in enumerate(slots):
        sc, gi = sl["splats"].c(), sl["g_in"].c()
        acc, gout = list(sl["acc"]), list(sl["g_out"])
        status = sl.get("status") or [None] * len(acc)
        if not (len(acc) == len(gout) == len(status)) or not 1 <= len(acc) <= _lib.TG_MAX_FRAMES:
            raise ValueError("acc, g_out and status need one entry per frame, 1..TG_MAX_FRAMES frames")
        gos = [g.c() for g in gout]
        keep += [sc, gi, gos]
        arr[i].s = ctypes.addressof(sc)
        arr[i].g_in = ctypes.addressof(gi)
        arr[i].cams = _addr(sl["cams"])
        arr[i].N = int(sl["n"])
        arr[i].V = int(sl["V"])
        arr[i].F = len(acc)
        for f in range(len(acc)):
            arr[i].acc[f] = _addr(acc[f])
            arr[i].g_out[f] = ctypes.addressof(gos[f])
            arr[i].status[f] = _addr(status[f])
    check("tg_solve_triangulate_batch", lib().tg_solve_triangulate_batch(arr, len(slots), ctypes.byref(params),
                                                                         stream_ptr(stream)))
    del keep


def bin_expand(s: SplatTensors, bins: BinTensors, n, cams, params, stream=None):
    """Per-tile depth-ordered lists (tile_ids, tile_ranges [T,2]); syncs."""
    cams = cams if isinstance(cams, ctypes.Array) else _lib.cameras(cams)
    L = lib()
    T = L.tg_num_tiles(cams, len(cams))
    sc, bc = s.c(), bins.c()
    nb = ctypes.c_size_t(0)
    check("tg_bin_expand", L.tg_bin_expand(ctypes.byref(sc), ctypes.byref(bc), n, cams, len(cams),
                                           ctypes.byref(params), None, None, 0, None, None, ctypes.byref(nb), None))
    dev = s.rec.device
    ws = torch.empty(int(nb.value), dtype=torch.uint8, device=dev)
    ranges = torch.empty(T, 2, dtype=torch.int32, device=dev)
    n_out = torch.zeros(1, dtype=torch.int64, device=dev)
    cap = max(int(bins.capacity) * 64, 1)
    for _ in range(2):
        ids = torch.empty(cap, dtype=torch.int32, device=dev)
        check("tg_bin_expand", L.tg_bin_expand(ctypes.byref(sc), ctypes.byref(bc), n, cams, len(cams),
                                               ctypes.byref(params), _ptr(ids), _ptr(ranges), cap, _ptr(n_out),
                                               _ptr(ws), ctypes.byref(nb), stream_ptr(stream)))
        torch.cuda.synchronize()
        tot = int(n_out.item())
        if tot <= cap:
            return ids[:tot], ranges
        cap = tot
    raise RuntimeError("tg_bin_expand: capacity did not converge")


# ---------------------------------------------------------------- frame object
class MotionTransfer:
    """Buffers and calls for one frame of motion transfer (N Gaussians, V
    views of one resolution).  All work is queued on the current stream."""

    def __init__(self, cams, n, device="cuda", params=None, capacity=None):
        self.cams_host = cams if isinstance(cams, ctypes.Array) else _lib.cameras(cams)
        self.V = len(self.cams_host)
        self.N = int(n)
        self.W = int(self.cams_host[0].width)
        self.H = int(self.cams_host[0].height)
        self.device = torch.device(device)
        self.params = params if params is not None else _lib.default_params()
        L = lib()
        self.n_cells = int(L.tg_num_cells(self.cams_host, self.V, self.N, ctypes.byref(self.params)))
        if self.n_cells < 0:
            raise ValueError("unsupported camera set")
        self.splats = SplatTensors.alloc(self.V, self.N, self.device)
        if capacity is None:
            capacity = max(1024, 4 * self.N * self.V)
        self._alloc_bins(capacity)
        VN = (self.V, self.N)
        self.acc = torch.empty(*VN, 16, dtype=torch.float32, device=self.device)
        self.mu_new = torch.empty(*VN, 2, dtype=torch.float32, device=self.device)
        self.cov_new = torch.empty(*VN, 3, dtype=torch.float32, device=self.device)
        self.vflags = torch.empty(*VN, dtype=torch.uint8, device=self.device)
        self.wn = torch.empty(*VN, 2, dtype=torch.float32, device=self.device)
        self.status = torch.empty(self.N, dtype=torch.int32, device=self.device)
        self.t_final = None
        self.stats = torch.zeros(4, dtype=torch.int64, device=self.device)

    def _alloc_bins(self, capacity):
        self.bins = BinTensors.alloc(self.V, self.N, self.n_cells, capacity, self.device)
        nb = bin_sort_ws_bytes(self.N, self.cams_host, self.params, capacity)
        self.ws = torch.empty(nb, dtype=torch.uint8, device=self.device)

    # -- stages
    def preprocess(self, g: GaussianTensors):
        preprocess(g, self.cams_host, self.params, self.splats)

    def bin_sort(self, check_overflow=True):
        bin_sort(self.splats, self.N, self.cams_host, self.params, self.bins, self.ws)
        if check_overflow:
            torch.cuda.current_stream().synchronize()
            if int(self.bins.overflow.item()):
                need = int(self.bins.n_pairs.item())
                self._alloc_bins(int(need * 1.1) + 1024)
                bin_sort(self.splats, self.N, self.cams_host, self.params, self.bins, self.ws)

    def accumulate(self, disp, vis=None, t_final=False, stats=False):
        acc_zero(self.acc)
        if t_final and self.t_final is None:
            self.t_final = torch.empty(self.V, self.H, self.W, dtype=torch.float32, device=self.device)
        if stats:
            self.stats.zero_()
        splat_accumulate(self.splats, self.bins, self.N, self.cams_host, disp, vis, self.params, self.acc,
                         self.t_final if t_final else None, self.stats if stats else None)

    def solve(self):
        solve_views(self.acc, self.splats, self.N, self.V, self.params, self.mu_new, self.cov_new, self.vflags,
                    self.wn)

    def triangulate(self, g_in: GaussianTensors, g_out: GaussianTensors):
        triangulate(self.mu_new, self.cov_new, self.vflags, self.wn, self.splats, g_in, self.cams_host,
                    self.params, g_out, self.status)

    def update(self, g_in: GaussianTensors, g_out: GaussianTensors):
        """Fused per-view solve + multi-view update (tg_solve_triangulate)."""
        solve_triangulate(self.acc, self.splats, g_in, self.cams_host, self.params, g_out, self.status)

    def run(self, g: GaussianTensors, disp, vis=None, g_out: GaussianTensors | None = None, check_overflow=True,
            t_final=False, stats=False, fused=False):
        """Cold frame: preprocess -> bin_sort -> accumulate -> solve ->
        triangulate (fused: the last two in one launch)."""
        if g_out is None:
            g_out = GaussianTensors(torch.empty_like(g.means), torch.empty_like(g.quats),
                                    torch.empty_like(g.scales), g.opacity, g.sh, g.sh_degree, g.scale_mode,
                                    g.opacity_mode)
        self.preprocess(g)
        self.bin_sort(check_overflow=check_overflow)
        self.accumulate(disp, vis, t_final=t_final, stats=stats)
        if fused:
            self.update(g, g_out)
        else:
            self.solve()
            self.triangulate(g, g_out)
        return g_out

    def run_warm(self, g: GaussianTensors, disp, vis, g_out: GaussianTensors):
        """Warm frame (splats and bins of the reference frame resident)."""
        self.accumulate(disp, vis)
        self.update(g, g_out)
        return g_out
