"""Python API over libpt: torch tensors hold device memory, the torch current
stream is the HIP stream.  Every computation runs in libpt's HIP kernels."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import capi
from .capi import check, lib


def _stream_handle(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _require_cuda(device):
    if not torch.cuda.is_available():
        raise RuntimeError("a ROCm GPU is required (libpt has no CPU path)")
    return torch.device(device)


def camera_struct(cam: dict) -> capi.Camera:
    c = capi.Camera()
    c.pos[:] = [float(v) for v in cam["pos"]]
    c.look_at[:] = [float(v) for v in cam["look_at"]]
    c.up[:] = [float(v) for v in cam["up"]]
    c.vfov_deg = float(cam["vfov"])
    return c


# pt_group.traversal by name
TRAVERSALS = {"auto": 0, "pair": 1, "wide": 2, "queue": 3, "quant": 4}


def group_struct(tile=(8, 8), k=8, reuse_max_bounce=0xFFFF, refill=0, waves_per_cu=0, leaf_gate=0,
                 nee=False, traversal=0, frame_groups=False) -> capi.Group:
    g = capi.Group()
    g.tile_w, g.tile_h = int(tile[0]), int(tile[1])
    g.k = int(k)
    g.reuse_max_bounce = int(min(reuse_max_bounce, 0xFFFF))
    g.refill = int(refill)
    g.waves_per_cu = int(waves_per_cu)
    g.leaf_gate = int(leaf_gate)
    g.nee = int(bool(nee))
    g.traversal = TRAVERSALS[traversal] if isinstance(traversal, str) else int(traversal)
    g.frame_groups = int(bool(frame_groups))
    return g


class Scene:
    """A scene built (BVH on the host) and uploaded into a torch-owned device arena."""

    def __init__(self, scene: dict, device="cuda:0", upload: bool = True):
        self.desc_src = scene
        self._tris = np.ascontiguousarray(scene["tris"], dtype=np.float32)
        self._mat = np.ascontiguousarray(scene["tri_mat"], dtype=np.uint32)
        self._mats = np.ascontiguousarray(scene["mats"])
        assert self._mats.dtype.itemsize == C.sizeof(capi.Material)
        d = capi.SceneDesc()
        d.tris = self._tris.ctypes.data
        d.ntri = int(self._tris.shape[0])
        d.tri_mat = self._mat.ctypes.data
        d.mats = self._mats.ctypes.data
        d.nmat = len(self._mats)
        d.env_radiance[:] = [float(v) for v in scene["env"]]
        h = C.c_void_p()
        check(lib().pt_scene_create(C.byref(d), C.byref(h)))
        self.handle = h
        self.camera = scene.get("camera")
        self.arena = None
        self.device = None
        if upload:
            self.upload(device)

    def upload(self, device="cuda:0"):
        dev = _require_cuda(device)
        nbytes = lib().pt_scene_device_bytes(self.handle)
        with torch.cuda.device(dev):
            self.arena = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=dev)
            assert self.arena.data_ptr() % 256 == 0
            check(lib().pt_scene_upload(self.handle, self.arena.data_ptr(), self.arena.numel(),
                                        _stream_handle(dev)))
        self.device = dev
        return self

    def info(self) -> dict:
        i = capi.SceneInfo()
        check(lib().pt_scene_get_info(self.handle, C.byref(i)))
        return dict(ntri=i.ntri, nnodes=i.nnodes, max_depth=i.max_depth, max_leaf=i.max_leaf,
                    lo=list(i.lo), hi=list(i.hi), sah_cost=i.sah_cost, device_bytes=i.device_bytes, nemit=i.nemit,
                    nnodes4=i.nnodes4, max_depth4=i.max_depth4, wide=i.wide, quant=i.quant)

    def export_bvh(self):
        inf = self.info()
        nodes = np.zeros((inf["nnodes"], 16), dtype=np.float32)
        order = np.zeros(inf["ntri"], dtype=np.uint32)
        check(lib().pt_scene_export_bvh(self.handle, nodes.ctypes.data, order.ctypes.data))
        return nodes, order

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                lib().pt_scene_free(h)
            except Exception:
                pass
            self.handle = None


class Timer:
    def __init__(self, capacity: int = 4096):
        h = C.c_void_p()
        check(lib().pt_timer_create(int(capacity), C.byref(h)))
        self.handle = h
        self.capacity = capacity

    def reset(self):
        check(lib().pt_timer_reset(self.handle))

    def read(self):
        n = C.c_int32()
        ms = np.zeros(self.capacity, np.float32)
        kind = np.zeros(self.capacity, np.int32)
        bounce = np.zeros(self.capacity, np.int32)
        check(lib().pt_timer_read(self.handle, ms.ctypes.data, kind.ctypes.data, bounce.ctypes.data,
                                  self.capacity, C.byref(n)))
        m = n.value
        return ms[:m], kind[:m], bounce[:m]

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                lib().pt_timer_free(h)
            except Exception:
                pass
            self.handle = None


@dataclass
class RenderConfig:
    w: int
    h: int
    spp: int = 1
    bounces: int = 2
    mode: str = "incoherent"
    tile: tuple = (8, 8)
    k: int = 8
    reuse_max_bounce: int | None = None
    refill: int = 0
    waves_per_cu: int = 0
    leaf_gate: int = 0
    nee: bool = False
    traversal: int | str = 0
    frame_groups: bool = False


class Renderer:
    """Holds the workspace and output tensors for repeated frames of one configuration."""

    def __init__(self, scene: Scene, cfg: RenderConfig, stats: bool = False, timer: Timer | None = None,
                 rays: bool = False, touched: bool = False, debug: bool = False):
        self.scene = scene
        self.cfg = cfg
        dev = scene.device
        B = cfg.bounces
        rmax = B if cfg.reuse_max_bounce is None else cfg.reuse_max_bounce
        self.group = group_struct(cfg.tile, cfg.k, rmax, cfg.refill, cfg.waves_per_cu, cfg.leaf_gate, cfg.nee,
                                  cfg.traversal, cfg.frame_groups)
        self.mode = capi.MODES[cfg.mode]
        ws = lib().pt_render_workspace_bytes(cfg.w, cfg.h, cfg.spp, B, self.mode, self.group)
        if ws == 0:
            raise capi.PtError(capi.PT_EINVAL, "invalid render configuration")
        with torch.cuda.device(dev):
            self.workspace = torch.empty(ws, dtype=torch.uint8, device=dev)
            self.radiance = torch.empty((cfg.h, cfg.w, 3), dtype=torch.float32, device=dev)
            self.hit_prim = torch.empty((B + 1, cfg.spp, cfg.h, cfg.w), dtype=torch.int32, device=dev)
            self.hit_t = torch.empty((B + 1, cfg.spp, cfg.h, cfg.w), dtype=torch.float32, device=dev)
            self.ray_count = torch.empty((B + 1, cfg.spp), dtype=torch.int32, device=dev)
            self.shadow_count = torch.empty((B + 1, cfg.spp), dtype=torch.int32, device=dev) if cfg.nee else None
            self.stats = torch.empty((B + 1, 2), dtype=torch.int64, device=dev) if stats else None
            inf = scene.info()
            self.touched = (torch.zeros(inf["nnodes"] + inf["ntri"], dtype=torch.uint8, device=dev)
                            if (stats and touched) else None)
            self.rays = torch.zeros((B + 1, cfg.spp, cfg.h, cfg.w, 8), dtype=torch.float32, device=dev) if rays else None
            self.debug = (torch.zeros((max(B, 1), cfg.spp, cfg.h, cfg.w, 4), dtype=torch.float32, device=dev)
                          if debug else None)
        self.timer = timer
        self.out = capi.Outputs()
        self.out.radiance = self.radiance.data_ptr()
        self.out.hit_prim = self.hit_prim.data_ptr()
        self.out.hit_t = self.hit_t.data_ptr()
        self.out.ray_count = self.ray_count.data_ptr()
        self.out.stats = self.stats.data_ptr() if stats else None
        self.out.rays = self.rays.data_ptr() if rays else None
        self.out.timer = timer.handle if timer is not None else None
        self.out.shadow_count = self.shadow_count.data_ptr() if cfg.nee else None
        self.out.touched = self.touched.data_ptr() if self.touched is not None else None
        self.out.debug = self.debug.data_ptr() if self.debug is not None else None

    def render(self, seed: int = 1, camera: dict | None = None):
        cfg = self.cfg
        cam = camera_struct(camera or self.scene.camera)
        dev = self.scene.device
        with torch.cuda.device(dev):
            check(lib().pt_render(self.scene.handle, C.byref(cam), cfg.w, cfg.h, cfg.spp, cfg.bounces,
                                  self.mode, self.group, C.c_uint64(int(seed)), self.workspace.data_ptr(),
                                  self.workspace.numel(), C.byref(self.out), _stream_handle(dev)))
        return self

    def results(self) -> dict:
        r = dict(radiance=self.radiance, hit_prim=self.hit_prim, hit_t=self.hit_t,
                 rays_per_bounce=self.ray_count.sum(dim=1))
        if self.stats is not None:
            r["stats"] = self.stats
        if self.rays is not None:
            r["rays"] = self.rays
        if self.shadow_count is not None:
            r["shadow_rays_per_bounce"] = self.shadow_count.sum(dim=1)
        if self.touched is not None:
            r["touched"] = self.touched
        if self.debug is not None:
            r["debug"] = self.debug
        return r

    def touched_counts(self) -> tuple:
        """Distinct nodes and triangles the traversal of each bounce b < 8 touched (sample 0) in
        the frames rendered since the flags were cleared: two int arrays of length B + 1."""
        assert self.touched is not None, "Renderer(..., stats=True, touched=True)"
        nn = self.scene.info()["nnodes"]
        B = self.cfg.bounces
        t = self.touched.to(torch.int32)
        bits = torch.tensor([1 << b for b in range(min(B + 1, 8))], dtype=torch.int32, device=t.device)
        hit = (t[None, :] & bits[:, None]) != 0
        nodes = hit[:, :nn].sum(dim=1).cpu().numpy()
        tris = hit[:, nn:].sum(dim=1).cpu().numpy()
        return nodes, tris


def render(scene: Scene, w, h, spp=1, bounces=2, mode="incoherent", tile=(8, 8), k=8,
           reuse_max_bounce=None, seed=1, camera=None, stats=False, rays=False, refill=0, leaf_gate=0,
           nee=False, traversal=0, frame_groups=False, debug=False) -> dict:
    r = Renderer(scene, RenderConfig(w, h, spp, bounces, mode, tuple(tile), k, reuse_max_bounce, refill, 0, leaf_gate,
                                     nee, traversal, frame_groups), stats=stats, rays=rays, debug=debug)
    r.render(seed, camera)
    return r.results()


def trace(scene: Scene, rays: torch.Tensor, refill: int = 0):
    """rays: device float32 [n, 8]; returns (prim int32 [n], t float32 [n])."""
    assert rays.dtype == torch.float32 and rays.is_contiguous() and rays.shape[-1] == 8
    dev = scene.device
    n = rays.shape[0]
    prim = torch.empty(n, dtype=torch.int32, device=dev)
    t = torch.empty(n, dtype=torch.float32, device=dev)
    ws = torch.empty(lib().pt_trace_workspace_bytes(), dtype=torch.uint8, device=dev)
    with torch.cuda.device(dev):
        check(lib().pt_trace(scene.handle, rays.data_ptr(), n, int(refill), prim.data_ptr(), t.data_ptr(), ws.data_ptr(),
                             ws.numel(), _stream_handle(dev)))
    return prim, t


def trace_static(scene: Scene, rays: torch.Tensor, refill: int = 0, waves_per_cu: int = 0):
    """pt_trace_static: as trace(), with the library's fixed scratch instead of a workspace."""
    assert rays.dtype == torch.float32 and rays.is_contiguous() and rays.shape[-1] == 8
    dev = scene.device
    n = rays.shape[0]
    prim = torch.empty(n, dtype=torch.int32, device=dev)
    t = torch.empty(n, dtype=torch.float32, device=dev)
    with torch.cuda.device(dev):
        check(lib().pt_trace_static(scene.handle, rays.data_ptr(), n, int(refill), int(waves_per_cu), prim.data_ptr(),
                                    t.data_ptr(), _stream_handle(dev)))
    return prim, t


def ray_keys(scene: Scene, rays: torch.Tensor, mode: str = "sorted") -> torch.Tensor:
    """Reordering keys of a sorted mode ("sorted" = TwoPoint, "sorted_origin", "sorted_reis",
    "sorted_aila"); int32 tensor holding the uint32 keys."""
    assert rays.dtype == torch.float32 and rays.is_contiguous() and rays.shape[-1] == 8
    dev = scene.device
    keys = torch.empty(rays.shape[0], dtype=torch.int32, device=dev)
    with torch.cuda.device(dev):
        check(lib().pt_ray_keys(scene.handle, rays.data_ptr(), rays.shape[0], capi.MODES[mode], keys.data_ptr(),
                                _stream_handle(dev)))
    return keys


def sort_pairs(keys: torch.Tensor, vals: torch.Tensor):
    """In-place stable sort of (keys, vals) by the 32-bit key (int32 tensors viewed as uint32)."""
    assert keys.dtype == torch.int32 and vals.dtype == torch.int32 and keys.numel() == vals.numel()
    dev = keys.device
    n = keys.numel()
    ws = torch.empty(max(lib().pt_sort_workspace_bytes(n), 256), dtype=torch.uint8, device=dev)
    with torch.cuda.device(dev):
        check(lib().pt_sort_pairs(keys.data_ptr(), vals.data_ptr(), n, ws.data_ptr(), ws.numel(),
                                  _stream_handle(dev)))
    return keys, vals


def probe_memory(nbytes: int, passes: int, chase_steps: int, buf: "torch.Tensor | None" = None,
                 device="cuda:0") -> dict:
    """Read bandwidth (GB/s) and dependent-load latency (ns) of the memory level that
    holds a buffer of nbytes (pt_probe_memory); buf: optional scratch of >= nbytes."""
    dev = _require_cuda(device)
    with torch.cuda.device(dev):
        if buf is None:
            buf = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        assert buf.numel() >= nbytes
        g, ns = C.c_float(), C.c_float()
        check(lib().pt_probe_memory(buf.data_ptr(), int(nbytes), int(passes), int(chase_steps), C.byref(g),
                                    C.byref(ns), _stream_handle(dev)))
    return dict(bytes=int(nbytes), read_gbps=g.value, chase_ns=ns.value)


def device_info():
    cu, ma, mi = C.c_int32(), C.c_int32(), C.c_int32()
    check(lib().pt_device_info(C.byref(cu), C.byref(ma), C.byref(mi)))
    return dict(compute_units=cu.value, major=ma.value, minor=mi.value)


class JobOutputs:
    """Device outputs of one batched job (torch tensors)."""

    def __init__(self, w, h, spp, bounces, device):
        self.radiance = torch.empty((h, w, 3), dtype=torch.float32, device=device)
        self.hit_prim = torch.empty((bounces + 1, spp, h, w), dtype=torch.int32, device=device)
        self.hit_t = torch.empty((bounces + 1, spp, h, w), dtype=torch.float32, device=device)

    @property
    def nbytes(self):
        return sum(t.numel() * t.element_size() for t in (self.radiance, self.hit_prim, self.hit_t))


def batch_job_bytes(w, h, spp, bounces, mode, tile=(8, 8), k=8, refill=0, waves_per_cu=0, leaf_gate=0) -> int:
    """Arena bytes one job of this shape takes in a batch (pt_batch_job_bytes)."""
    j = capi.Job()
    j.w, j.h, j.spp, j.bounces = int(w), int(h), int(spp), int(bounces)
    j.mode = capi.MODES[mode]
    n = int(lib().pt_batch_job_bytes(C.byref(j), group_struct(tile, k, 0xFFFF, refill, waves_per_cu, leaf_gate)))
    if n == 0:
        raise capi.PtError(capi.PT_EINVAL, "invalid job shape")
    return n


class Batch:
    """Jobs in flight over device-resident scenes; merged launches per step (pt_batch_*)."""

    def __init__(self, max_jobs: int, arena_bytes: int, tile=(8, 8), k=8, reuse_max_bounce=0xFFFF, refill=0,
                 waves_per_cu=0, leaf_gate=0, device="cuda:0", traversal=0, frame_groups=False):
        self.device = _require_cuda(device)
        self.group = group_struct(tile, k, reuse_max_bounce, refill, waves_per_cu, leaf_gate, traversal=traversal,
                                  frame_groups=frame_groups)
        base = lib().pt_batch_base_bytes(int(max_jobs))
        if base == 0:
            raise capi.PtError(capi.PT_EINVAL, "bad max_jobs")
        with torch.cuda.device(self.device):
            self.arena = torch.empty(max(int(arena_bytes), base), dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        check(lib().pt_batch_create(int(max_jobs), self.group, self.arena.data_ptr(), self.arena.numel(), C.byref(h)))
        self.handle = h
        self.jobs = {}

    @staticmethod
    def base_bytes(max_jobs: int) -> int:
        return int(lib().pt_batch_base_bytes(int(max_jobs)))

    def job_struct(self, scene: Scene, w, h, spp, bounces, mode, seed, out: JobOutputs, camera=None) -> capi.Job:
        j = capi.Job()
        j.scene = scene.handle.value
        j.camera = camera_struct(camera or scene.camera)
        j.w, j.h, j.spp, j.bounces = int(w), int(h), int(spp), int(bounces)
        j.mode = capi.MODES[mode]
        j.seed = int(seed)
        j.radiance, j.hit_prim, j.hit_t = out.radiance.data_ptr(), out.hit_prim.data_ptr(), out.hit_t.data_ptr()
        return j

    def job_bytes(self, job: capi.Job) -> int:
        return int(lib().pt_batch_job_bytes(C.byref(job), self.group))

    def submit(self, job: capi.Job, keep=None):
        """Returns the job id, or None when the batch is full (PT_EBUSY)."""
        jid = C.c_uint32()
        st = lib().pt_batch_submit(self.handle, C.byref(job), C.byref(jid))
        if st == capi.PT_EBUSY:
            return None
        check(st)
        self.jobs[jid.value] = (job, keep)
        return jid.value

    def step(self) -> int:
        active = C.c_int32()
        with torch.cuda.device(self.device):
            check(lib().pt_batch_step(self.handle, _stream_handle(self.device), C.byref(active)))
        return active.value

    def done(self, jid: int) -> bool:
        d = C.c_int32()
        check(lib().pt_batch_poll(self.handle, int(jid), C.byref(d)))
        return bool(d.value)

    def release(self, jid: int):
        check(lib().pt_batch_release(self.handle, int(jid)))
        self.jobs.pop(jid, None)

    def run(self, use_graph: bool = False, timer: "Timer | None" = None):
        with torch.cuda.device(self.device):
            check(lib().pt_batch_run(self.handle, int(bool(use_graph)), timer.handle if timer else None,
                                     _stream_handle(self.device)))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                torch.cuda.synchronize(self.device)
                lib().pt_batch_free(h)
            except Exception:
                pass
            self.handle = None
