"""ctypes binding of the CPU oracle.

TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import this; the GPU product path never does.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import LIB as _BUILT_LIB, build

# PT_ORACLE_LIB names another build of the oracle (the mutation test loads
# deliberately broken copies this way); default: the library oracle/build.py makes
LIB = os.environ.get("PT_ORACLE_LIB") or _BUILT_LIB

MODE = {"incoherent": 0, "sorted": 1, "reuse": 2, "sorted_origin": 3, "sorted_reis": 4, "sorted_aila": 5,
        "reuse_plain": 6, "reuse_world": 7}

F_ACTIVE = 1 << 0
F_CLASS_SH = 1
F_CAT_SH = 3
F_REP = 1 << 5
F_REUSED = 1 << 6
F_VALID = 1 << 7
F_SLOT_SH = 16


class _Material(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("albedo", C.c_float * 3), ("alpha", C.c_float),
                ("emission", C.c_float * 3)]


class _Camera(C.Structure):
    _fields_ = [("pos", C.c_float * 3), ("look_at", C.c_float * 3), ("up", C.c_float * 3),
                ("vfov_deg", C.c_float)]


class _Outputs(C.Structure):
    _fields_ = [("radiance", C.c_void_p), ("hit_prim", C.c_void_p), ("hit_t", C.c_void_p),
                ("hit_t2", C.c_void_p), ("dbg_q", C.c_void_p), ("dbg_flags", C.c_void_p),
                ("dbg_keys", C.c_void_p), ("rays", C.c_void_p), ("rays_per_bounce", C.c_void_p),
                ("shadow_rays", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            if LIB != _BUILT_LIB:
                raise FileNotFoundError(LIB)
            build()
        L = C.CDLL(LIB)
        vp, u32, i32, f = C.c_void_p, C.c_uint32, C.c_int, C.c_float
        L.orc_scene_create.restype = vp
        L.orc_scene_create.argtypes = [vp, u32, vp, vp, u32, vp]
        L.orc_scene_free.argtypes = [vp]
        L.orc_scene_bounds.argtypes = [vp, vp, vp]
        L.orc_trace.argtypes = [vp, vp, u32, vp, vp, vp, vp, vp]
        L.orc_trace_brute.argtypes = [vp, vp, u32, vp, vp]
        L.orc_render.restype = i32
        L.orc_render.argtypes = [vp, vp, i32, i32, i32, i32, i32, i32, i32, i32, i32, i32, C.c_uint64, vp, i32, vp]
        L.orc_philox4x64_10.argtypes = [vp, vp, vp]
        L.orc_sincos2pi.argtypes = [vp, u32, vp, vp]
        L.orc_onb.argtypes = [vp, vp, vp]
        L.orc_sample_lambert.argtypes = [f, f, vp]
        L.orc_sample_ggx.restype = i32
        L.orc_sample_ggx.argtypes = [vp, f, vp, f, f, vp, vp]
        L.orc_offset_origin.argtypes = [vp, vp, vp]
        L.orc_shuffle.argtypes = [i32, C.c_uint64, C.c_uint64, vp]
        L.orc_ray_key.restype = u32
        L.orc_ray_key.argtypes = [vp, vp, vp, vp]
        L.orc_ray_key_kind.restype = u32
        L.orc_ray_key_kind.argtypes = [C.c_int, vp, vp, vp, vp]
        L.orc_camera_ray.argtypes = [vp, i32, i32, i32, i32, f, f, vp, vp]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def camera_struct(cam: dict) -> _Camera:
    c = _Camera()
    c.pos[:] = [float(v) for v in cam["pos"]]
    c.look_at[:] = [float(v) for v in cam["look_at"]]
    c.up[:] = [float(v) for v in cam["up"]]
    c.vfov_deg = float(cam["vfov"])
    return c


class OracleScene:
    def __init__(self, scene: dict):
        self.scene = scene
        self._tris = np.ascontiguousarray(scene["tris"], dtype=np.float32)
        self._mat = np.ascontiguousarray(scene["tri_mat"], dtype=np.uint32)
        self._mats = np.ascontiguousarray(scene["mats"])
        assert self._mats.dtype.itemsize == 32
        self._env = np.ascontiguousarray(scene["env"], dtype=np.float32)
        self.ntri = int(self._tris.shape[0])
        self.h = lib().orc_scene_create(_p(self._tris), self.ntri, _p(self._mat), _p(self._mats),
                                        len(self._mats), _p(self._env))
        if not self.h:
            raise MemoryError("oracle scene allocation failed")
        self._free = lib().orc_scene_free   # held here: module globals may be gone at interpreter exit

    def __del__(self):
        if getattr(self, "h", None) and getattr(self, "_free", None):
            self._free(self.h)
            self.h = None

    def bounds(self):
        lo = np.zeros(3, np.float32)
        hi = np.zeros(3, np.float32)
        lib().orc_scene_bounds(self.h, _p(lo), _p(hi))
        return lo, hi

    def trace(self, rays: np.ndarray, stats: bool = False):
        rays = np.ascontiguousarray(rays, dtype=np.float32).reshape(-1, 8)
        n = rays.shape[0]
        prim = np.empty(n, np.int32)
        t = np.empty(n, np.float32)
        t2 = np.empty(n, np.float32)
        nv = np.zeros(1, np.uint64)
        nt = np.zeros(1, np.uint64)
        lib().orc_trace(self.h, _p(rays), n, _p(prim), _p(t), _p(t2), _p(nv), _p(nt))
        if stats:
            return prim, t, t2, int(nv[0]), int(nt[0])
        return prim, t, t2

    def trace_brute(self, rays: np.ndarray):
        rays = np.ascontiguousarray(rays, dtype=np.float32).reshape(-1, 8)
        n = rays.shape[0]
        prim = np.empty(n, np.int32)
        t = np.empty(n, np.float32)
        lib().orc_trace_brute(self.h, _p(rays), n, _p(prim), _p(t))
        return prim, t

    def render(self, w, h, spp, bounces, mode="incoherent", tile=(8, 8), k=8, reuse_max_bounce=None,
               seed=1, tile_mask=None, debug=False, camera=None, nee=False, rays=False, frame_groups=False):
        cam = camera_struct(camera or self.scene["camera"])
        B = int(bounces)
        if reuse_max_bounce is None:
            reuse_max_bounce = B
        rad = np.zeros((h, w, 3), np.float32)
        hp = np.full((B + 1, spp, h, w), -2, np.int32)
        ht = np.full((B + 1, spp, h, w), np.inf, np.float32)
        ht2 = np.full((B + 1, spp, h, w), np.inf, np.float32)
        rpb = np.zeros(B + 1, np.uint64)
        srb = np.zeros(B + 1, np.uint64)
        out = _Outputs()
        out.radiance, out.hit_prim, out.hit_t, out.hit_t2 = _p(rad), _p(hp), _p(ht), _p(ht2)
        out.rays_per_bounce = _p(rpb)
        out.shadow_rays = _p(srb)
        res = dict(radiance=rad, hit_prim=hp, hit_t=ht, hit_t2=ht2, rays_per_bounce=rpb, shadow_rays=srb)
        if debug:
            q = np.zeros((max(B, 1), spp, h, w, 3), np.float32)
            fl = np.zeros((max(B, 1), spp, h, w), np.int32)
            keys = np.full((max(B, 1), spp, h, w), 0xFFFFFFFF, np.uint32)
            rays = np.zeros((B + 1, spp, h, w, 8), np.float32)
            out.dbg_q, out.dbg_flags, out.dbg_keys, out.rays = _p(q), _p(fl), _p(keys), _p(rays)
            res.update(dbg_q=q[:B], dbg_flags=fl[:B], dbg_keys=keys[:B], rays=rays)
        elif rays:
            rr = np.zeros((B + 1, spp, h, w, 8), np.float32)
            out.rays = _p(rr)
            res.update(rays=rr)
        mask = None
        if tile_mask is not None:
            mask = np.ascontiguousarray(tile_mask, dtype=np.uint8)
            ntx = (w + tile[0] - 1) // tile[0]
            nty = (h + tile[1] - 1) // tile[1]
            assert mask.size == ntx * nty
        rc = lib().orc_render(self.h, C.byref(cam), w, h, spp, B, MODE[mode], tile[0], tile[1], k,
                              int(reuse_max_bounce), int(bool(frame_groups)), C.c_uint64(seed), _p(mask),
                              int(bool(nee)), C.byref(out))
        if rc != 0:
            raise ValueError(f"orc_render failed with {rc}")
        return res


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    o = np.zeros(4, np.uint64)
    lib().orc_philox4x64_10(_p(c), _p(k), _p(o))
    return o


def sincos2pi(u: np.ndarray):
    u = np.ascontiguousarray(u, dtype=np.float32)
    s = np.empty_like(u)
    c = np.empty_like(u)
    lib().orc_sincos2pi(_p(u), u.size, _p(s), _p(c))
    return s, c


def onb(n):
    n = np.ascontiguousarray(n, dtype=np.float32)
    t = np.zeros(3, np.float32)
    b = np.zeros(3, np.float32)
    lib().orc_onb(_p(n), _p(t), _p(b))
    return t, b


def sample_lambert(u2, u3):
    q = np.zeros(3, np.float32)
    lib().orc_sample_lambert(float(u2), float(u3), _p(q))
    return q


def sample_ggx(wi, alpha, f0, u2, u3):
    wi = np.ascontiguousarray(wi, dtype=np.float32)
    f0 = np.ascontiguousarray(f0, dtype=np.float32)
    wo = np.zeros(3, np.float32)
    w = np.zeros(3, np.float32)
    ok = lib().orc_sample_ggx(_p(wi), float(alpha), _p(f0), float(u2), float(u3), _p(wo), _p(w))
    return bool(ok), wo, w


def offset_origin(p, n):
    p = np.ascontiguousarray(p, dtype=np.float32)
    n = np.ascontiguousarray(n, dtype=np.float32)
    o = np.zeros(3, np.float32)
    lib().orc_offset_origin(_p(p), _p(n), _p(o))
    return o


def shuffle(wh, x0, x1):
    s = np.zeros(wh, np.uint32)
    lib().orc_shuffle(int(wh), C.c_uint64(int(x0)), C.c_uint64(int(x1)), _p(s))
    return s


def ray_key(lo, hi, o, d, kind="sorted"):
    """Reordering key of one ray; kind = one of the sorted modes ("sorted" = TwoPoint)."""
    a = [np.ascontiguousarray(v, dtype=np.float32) for v in (lo, hi, o, d)]
    if kind == "sorted":
        return int(lib().orc_ray_key(*[_p(v) for v in a]))
    return int(lib().orc_ray_key_kind(MODE[kind], *[_p(v) for v in a]))


def camera_ray(cam: dict, w, h, x, y, u0, u1):
    c = camera_struct(cam)
    o = np.zeros(3, np.float32)
    d = np.zeros(3, np.float32)
    lib().orc_camera_ray(C.byref(c), w, h, x, y, float(u0), float(u1), _p(o), _p(d))
    return o, d


def pack_rays(o: np.ndarray, d: np.ndarray, exclude=None) -> np.ndarray:
    """[n][8] float32 rays {ox,oy,oz,exclude-bits,dx,dy,dz,0}."""
    n = o.shape[0]
    r = np.zeros((n, 8), np.float32)
    r[:, 0:3] = o
    r[:, 4:7] = d
    ex = np.full(n, -1, np.int32) if exclude is None else np.asarray(exclude, np.int32)
    r[:, 3] = ex.view(np.float32)
    return r
