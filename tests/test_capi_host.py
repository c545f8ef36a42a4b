"""Host-side checks of libpt (no GPU): exported symbols, argument checks,
workspace sizes, and the validity of the host BVH build."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2310_07182_amd import capi, scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(capi.LIB_PATH):
        from paper_2310_07182_amd import build
        build.build()
    return capi.lib()


def test_exports_every_declared_symbol(L):
    hdr = open(os.path.join(ROOT, "include", "pt.h")).read()
    decl = set(re.findall(r"^(?:pt_status|size_t|const char\*)\s+(pt_[a-z0-9_]+)\s*\(", hdr, re.M))
    assert len(decl) >= 18
    for name in sorted(decl):
        assert hasattr(L, name), name
    assert decl == set(capi.PROTOTYPES), decl ^ set(capi.PROTOTYPES)


def test_sortref_exports_every_declared_symbol():
    import ctypes

    from paper_2310_07182_amd import build as B

    hdr = open(os.path.join(ROOT, "include", "pt_sortref.h")).read()
    decl = set(re.findall(r"^int\s+(ptref_[a-z0-9_]+)\s*\(", hdr, re.M))
    assert decl == {"ptref_sort_workspace_bytes", "ptref_sort_pairs"}, decl
    L2 = ctypes.CDLL(B.SORTREF_LIB)
    for name in sorted(decl):
        assert hasattr(L2, name), name


def _desc(scene):
    tris = np.ascontiguousarray(scene["tris"], np.float32)
    mat = np.ascontiguousarray(scene["tri_mat"], np.uint32)
    mats = np.ascontiguousarray(scene["mats"])
    d = capi.SceneDesc()
    d.tris, d.ntri, d.tri_mat, d.mats, d.nmat = tris.ctypes.data, len(tris), mat.ctypes.data, mats.ctypes.data, len(mats)
    d.env_radiance[:] = [float(v) for v in scene["env"]]
    return d, (tris, mat, mats)


def _create(L, scene):
    d, keep = _desc(scene)
    h = C.c_void_p()
    st = L.pt_scene_create(C.byref(d), C.byref(h))
    return st, h, keep


def _bvh(L, h):
    info = capi.SceneInfo()
    assert L.pt_scene_get_info(h, C.byref(info)) == 0
    nodes = np.zeros((info.nnodes, 16), np.float32)
    order = np.zeros(info.ntri, np.uint32)
    assert L.pt_scene_export_bvh(h, nodes.ctypes.data, order.ctypes.data) == 0
    return info, nodes, order


def _check_bvh(tris, info, nodes, order):
    codes = nodes[:, 12:14].view(np.int32)
    assert np.array_equal(np.sort(order), np.arange(len(tris)))
    seen = np.zeros(len(tris), np.int32)
    EMPTY = np.iinfo(np.int32).min
    stack = [(0, 0)]
    max_depth = 0
    while stack:
        ni, depth = stack.pop()
        f = nodes[ni]
        boxes = [((f[0], f[2], f[8]), (f[1], f[3], f[9])), ((f[4], f[6], f[10]), (f[5], f[7], f[11]))]
        for c in range(2):
            code = int(codes[ni, c])
            if code == EMPTY:
                continue
            lo, hi = np.array(boxes[c][0]), np.array(boxes[c][1])
            if code >= 0:
                g = nodes[code]
                # the child's children lie inside the child's box
                for cc in range(2):
                    if int(codes[code, cc]) == EMPTY:
                        continue
                    glo = np.array([g[0 + 4 * cc], g[2 + 4 * cc], g[8 + 2 * cc]])
                    ghi = np.array([g[1 + 4 * cc], g[3 + 4 * cc], g[9 + 2 * cc]])
                    assert (glo >= lo).all() and (ghi <= hi).all()
                stack.append((code, depth + 1))
            else:
                v = ~code & 0xFFFFFFFF
                first, cnt = v >> 3, (v & 7) + 1
                assert cnt <= 4
                max_depth = max(max_depth, depth + 1)
                for j in range(first, first + cnt):
                    tv = tris[order[j]]
                    assert (tv.min(0) >= lo).all() and (tv.max(0) <= hi).all()
                    seen[order[j]] += 1
    assert (seen == 1).all()
    assert max_depth <= 64
    return max_depth


@pytest.mark.parametrize("fn", [scenes.tiny, scenes.furnace, scenes.mixed_small])
def test_bvh_valid(L, fn):
    s = fn()
    st, h, keep = _create(L, s)
    assert st == 0
    info, nodes, order = _bvh(L, h)
    assert info.ntri == len(s["tris"])
    assert np.allclose(info.lo, s["tris"].reshape(-1, 3).min(0)) and np.allclose(info.hi, s["tris"].reshape(-1, 3).max(0))
    _check_bvh(s["tris"], info, nodes, order)
    L.pt_scene_free(h)


def test_bvh_deterministic(L):
    s = scenes.mixed_small()
    outs = []
    for _ in range(2):
        st, h, keep = _create(L, s)
        info, nodes, order = _bvh(L, h)
        outs.append((nodes.copy(), order.copy()))
        L.pt_scene_free(h)
    assert np.array_equal(outs[0][0].view(np.uint32), outs[1][0].view(np.uint32))
    assert np.array_equal(outs[0][1], outs[1][1])


def test_bvh_degenerate_inputs(L):
    # all triangles identical (no SAH split possible) and tiny counts
    tri = np.array([[[0, 0, 0], [1, 0, 0], [0, 1, 0]]], np.float32)
    mats = np.array([(0, (0.5, 0.5, 0.5), 0.0, (0, 0, 0))], dtype=scenes.MATERIAL_DTYPE)
    for n in (1, 3, 4, 5, 37, 1000):
        s = dict(tris=np.repeat(tri, n, 0), tri_mat=np.zeros(n, np.uint32), mats=mats, env=np.ones(3, np.float32))
        st, h, keep = _create(L, s)
        assert st == 0
        info, nodes, order = _bvh(L, h)
        _check_bvh(s["tris"], info, nodes, order)
        L.pt_scene_free(h)


def test_empty_scene(L):
    mats = np.array([(0, (0.5, 0.5, 0.5), 0.0, (0, 0, 0))], dtype=scenes.MATERIAL_DTYPE)
    s = dict(tris=np.zeros((0, 3, 3), np.float32), tri_mat=np.zeros(0, np.uint32), mats=mats, env=np.ones(3, np.float32))
    st, h, keep = _create(L, s)
    assert st == 0
    info, nodes, order = _bvh(L, h)
    assert info.nnodes == 1 and info.ntri == 0
    L.pt_scene_free(h)


def test_scene_errors(L):
    s = scenes.furnace()
    bad = dict(s)
    bad["tri_mat"] = s["tri_mat"].copy()
    bad["tri_mat"][3] = 7
    st, h, keep = _create(L, bad)
    assert st == capi.PT_EINVAL and b"material" in L.pt_last_error()
    bad = dict(s)
    bad["tris"] = s["tris"].copy()
    bad["tris"][2, 1, 0] = np.nan
    st, h, keep = _create(L, bad)
    assert st == capi.PT_EINVAL and b"non-finite" in L.pt_last_error()
    assert L.pt_scene_create(None, None) == capi.PT_EINVAL


def _group(w, h, k, r=4):
    g = capi.Group()
    g.tile_w, g.tile_h, g.k, g.reuse_max_bounce = w, h, k, r
    return g


def test_workspace_sizes(L):
    ok = L.pt_render_workspace_bytes(1920, 1080, 1, 4, 2, _group(8, 8, 8))
    assert ok > 3 * 1920 * 1080 * 32
    srt = L.pt_render_workspace_bytes(1920, 1080, 1, 4, 1, _group(8, 8, 8))
    assert srt > ok
    for g in (_group(3, 4, 1), _group(8, 8, 3), _group(4, 4, 32), _group(64, 32, 8), _group(0, 8, 1)):
        assert L.pt_render_workspace_bytes(64, 64, 1, 2, 2, g) == 0
    assert L.pt_render_workspace_bytes(0, 64, 1, 2, 0, _group(4, 4, 2)) == 0
    assert L.pt_render_workspace_bytes(64, 64, 0, 2, 0, _group(4, 4, 2)) == 0
    assert L.pt_render_workspace_bytes(64, 64, 1, -1, 0, _group(4, 4, 2)) == 0
    assert L.pt_render_workspace_bytes(64, 64, 1, 0, 0, _group(32, 32, 1024)) > 0
    assert L.pt_sort_workspace_bytes(0) > 0 and L.pt_sort_workspace_bytes(10 ** 6) >= 8 * 10 ** 6
    assert L.pt_trace_workspace_bytes() > 0


def test_render_rejects_before_touching_device(L):
    s = scenes.furnace()
    st, h, keep = _create(L, s)
    cam = capi.Camera()
    out = capi.Outputs()
    # not uploaded
    st = L.pt_render(h, C.byref(cam), 8, 8, 1, 1, 0, _group(4, 4, 2), 1, None, 0, C.byref(out), None)
    assert st == capi.PT_EINVAL
    assert L.pt_render(None, C.byref(cam), 8, 8, 1, 1, 0, _group(4, 4, 2), 1, None, 0, C.byref(out), None) == capi.PT_EINVAL
    L.pt_scene_free(h)


def test_group_leaf_gate_checked(L):
    g = _group(8, 8, 8)
    g.leaf_gate = 65
    j = capi.Job()
    j.w, j.h, j.spp, j.bounces, j.mode = 64, 64, 1, 2, capi.MODES["reuse"]
    assert L.pt_batch_job_bytes(C.byref(j), g) == 0
    g.leaf_gate = 64
    assert L.pt_batch_job_bytes(C.byref(j), g) > 0


def test_batch_job_bytes_hold_queues_state_and_tile_flags(L):
    """A job's arena: two ray queues and the path state, 32 B per slot each (256-byte
    aligned), then one flag word per shade workgroup (one super tile of >= 64 slots)."""
    def al(x):
        return (x + 255) // 256 * 256
    j = capi.Job()
    for (w, h, tile, k) in ((1920, 1080, (8, 8), 8), (101, 67, (4, 4), 2), (70, 66, (32, 32), 128)):
        j.w, j.h, j.spp, j.bounces, j.mode = w, h, 1, 4, capi.MODES["reuse"]
        tw, th = tile
        if tw * th >= 64:
            sw, sh = tw, th
        else:
            cols = max(1, min(8 // tw, 64 // (tw * th)))
            sw, sh = cols * tw, (64 // (tw * th) // cols) * th
        nst = -(-w // sw) * -(-h // sh)
        nslots = nst * sw * sh
        assert L.pt_batch_job_bytes(C.byref(j), _group(tw, th, k)) == 3 * al(nslots * 32) + al(nst * 4)


def test_probe_rejects_before_touching_device(L):
    g, ns = C.c_float(), C.c_float()
    assert L.pt_probe_memory(None, 1 << 20, 1, 1, C.byref(g), C.byref(ns), None) == capi.PT_EINVAL
    assert L.pt_probe_memory(C.c_void_p(256), 1024, 1, 1, C.byref(g), C.byref(ns), None) == capi.PT_EINVAL
    assert L.pt_probe_memory(C.c_void_p(257), 1 << 20, 1, 1, C.byref(g), C.byref(ns), None) == capi.PT_EINVAL
    assert L.pt_probe_memory(C.c_void_p(256), 1 << 20, 0, 1, C.byref(g), C.byref(ns), None) == capi.PT_EINVAL
    assert L.pt_probe_memory(C.c_void_p(256), 1 << 20, 1, 1 << 25, C.byref(g), C.byref(ns), None) == capi.PT_EINVAL


def test_nee_checks(L):
    g = _group(8, 8, 8)
    g.nee = 2
    j = capi.Job()
    j.w, j.h, j.spp, j.bounces, j.mode = 64, 64, 1, 2, capi.MODES["reuse"]
    assert L.pt_batch_job_bytes(C.byref(j), g) == 0
    g.nee = 1
    assert L.pt_render_workspace_bytes(64, 64, 1, 2, capi.MODES["reuse"], g) > \
        L.pt_render_workspace_bytes(64, 64, 1, 2, capi.MODES["reuse"], _group(8, 8, 8))
    # batches refuse next-event estimation before touching the device
    h = C.c_void_p()
    assert L.pt_batch_create(4, g, C.c_void_p(1 << 20), 1 << 30, C.byref(h)) == capi.PT_EUNSUPPORTED


def test_scene_counts_emitters(L):
    s = scenes.mixed_small()
    st, h, keep = _create(L, s)
    assert st == capi.PT_OK
    info = capi.SceneInfo()
    assert L.pt_scene_get_info(h, C.byref(info)) == capi.PT_OK
    em = s["mats"]["emission"].max(axis=1) > 0
    assert info.nemit == int(em[s["tri_mat"]].sum()) > 0
    L.pt_scene_free(h)


def _bvh4(L, h):
    info = capi.SceneInfo()
    assert L.pt_scene_get_info(h, C.byref(info)) == 0
    raw = np.zeros((max(info.nnodes4, 1), 32), np.float32)
    assert L.pt_scene_export_bvh4(h, raw.ctypes.data) == 0
    return info, raw[: info.nnodes4]


@pytest.mark.parametrize("fn", [scenes.tiny, scenes.furnace, scenes.mixed_small, scenes.mid])
def test_bvh4_valid(L, fn):
    """The four-wide tree: every inner node is reached once, every child box holds its
    subtree, and the leaves cover every triangle exactly once."""
    s = fn()
    st, h, keep = _create(L, s)
    assert st == 0
    info, raw = _bvh4(L, h)
    nodes2, order = (lambda i: (i, None))(None)
    order = np.zeros(len(s["tris"]), np.uint32)
    info2 = capi.SceneInfo()
    L.pt_scene_get_info(h, C.byref(info2))
    n2 = np.zeros((info2.nnodes, 16), np.float32)
    L.pt_scene_export_bvh(h, n2.ctypes.data, order.ctypes.data)
    tris = np.asarray(s["tris"], np.float32).reshape(-1, 3, 3)
    boxes = raw[:, :24].reshape(-1, 6, 4)          # lx hx ly hy lz hz, x 4 children
    codes = raw[:, 24:28].view(np.int32)
    EMPTY = np.iinfo(np.int32).min
    seen_tri = np.zeros(len(tris), np.int32)
    seen_node = np.zeros(len(raw), np.int32)
    stack = [(0, 1)]
    max_depth = 0
    while stack:
        ni, depth = stack.pop()
        seen_node[ni] += 1
        max_depth = max(max_depth, depth)
        nchild = 0
        for c in range(4):
            code = int(codes[ni, c])
            if code == EMPTY:
                continue
            nchild += 1
            lo = np.array([boxes[ni, 0, c], boxes[ni, 2, c], boxes[ni, 4, c]])
            hi = np.array([boxes[ni, 1, c], boxes[ni, 3, c], boxes[ni, 5, c]])
            if code >= 0:
                assert 0 < code < len(raw)
                for cc in range(4):
                    if int(codes[code, cc]) == EMPTY:
                        continue
                    glo = np.array([boxes[code, 0, cc], boxes[code, 2, cc], boxes[code, 4, cc]])
                    ghi = np.array([boxes[code, 1, cc], boxes[code, 3, cc], boxes[code, 5, cc]])
                    assert (glo >= lo).all() and (ghi <= hi).all()
                stack.append((code, depth + 1))
            else:
                v = ~code & 0xFFFFFFFF
                first, cnt = v >> 3, (v & 7) + 1
                assert cnt <= 4 and first + cnt <= len(tris)
                for j in range(first, first + cnt):
                    tv = tris[order[j]]
                    assert (tv.min(0) >= lo).all() and (tv.max(0) <= hi).all()
                    seen_tri[order[j]] += 1
        assert nchild >= (1 if ni == 0 else 2)
    assert (seen_tri == 1).all()
    assert (seen_node == 1).all()
    assert max_depth == info.max_depth4
    assert info.nnodes4 < info2.nnodes
    assert info.wide == (1 if 3 * info.max_depth4 + 4 <= 80 else 0)
    L.pt_scene_free(h)


@pytest.mark.parametrize("fn,sample", [(scenes.tiny, None), (scenes.furnace, None), (scenes.mixed_small, 400),
                                       (scenes.mid, 300)])
def test_bvh4_quantized_boxes_enclose(L, fn, sample):
    """Quantized four-wide nodes: same codes as the four-wide nodes, and in exact
    arithmetic every child's quantized box p + q * 2^e encloses its float box; the steps
    are powers of two 2^e with -100 <= e <= 60 (so 2^e * inv stays a finite normal float)."""
    from fractions import Fraction
    s = fn()
    st, h, keep = _create(L, s)
    assert st == 0
    info, raw = _bvh4(L, h)
    q = np.zeros((max(info.nnodes4, 1), 16), np.uint32)
    assert L.pt_scene_export_bvh4q(h, q.ctypes.data) == 0
    q = q[: info.nnodes4]
    assert info.quant == 1
    assert np.array_equal(q[:, 4:8], raw[:, 24:28].view(np.uint32))
    boxes = raw[:, :24].reshape(-1, 6, 4).astype(np.float64)
    EMPTY = np.iinfo(np.int32).min
    codes = raw[:, 24:28].view(np.int32)
    idx = np.arange(len(q)) if sample is None else np.random.default_rng(5).choice(len(q), sample, replace=False)
    checked = 0
    for ni in idx:
        p = q[ni, :3].view(np.float32).astype(np.float64)
        steps = q[ni, [3, 14, 15]].view(np.float32).astype(np.float64)
        e = [int(np.log2(x)) for x in steps]
        assert all(-100 <= x <= 60 and 2.0 ** x == st for x, st in zip(e, steps))
        for c in range(4):
            planes = [(int(q[ni, 8 + 2 * a]) >> (8 * c)) & 0xFF for a in range(3)] + \
                     [(int(q[ni, 9 + 2 * a]) >> (8 * c)) & 0xFF for a in range(3)]
            if int(codes[ni, c]) == EMPTY:
                assert planes[:3] == [255] * 3 and planes[3:] == [0] * 3
                continue
            for a in range(3):
                step = Fraction(2) ** e[a]
                qlo = Fraction(p[a]) + planes[a] * step
                qhi = Fraction(p[a]) + planes[3 + a] * step
                assert qlo <= Fraction(boxes[ni, 2 * a, c]) and qhi >= Fraction(boxes[ni, 2 * a + 1, c])
                checked += 1
    assert checked > 0
    L.pt_scene_free(h)


def _shifted(s, offset, scale=1.0):
    out = dict(s)
    out["tris"] = np.ascontiguousarray((s["tris"].astype(np.float64) * scale + np.asarray(offset)).astype(np.float32))
    return out


def test_bvh4_quantized_far_from_origin(L):
    """A scene far from the origin (coordinates ~1e6, boxes of ~1 m): quantized boxes still
    enclose the float boxes exactly."""
    from fractions import Fraction
    s = _shifted(scenes.tiny(), (1.0e6, -3.0e5, 2.0e4))
    st, h, keep = _create(L, s)
    assert st == 0
    info, raw = _bvh4(L, h)
    assert info.quant == 1
    q = np.zeros((max(info.nnodes4, 1), 16), np.uint32)
    assert L.pt_scene_export_bvh4q(h, q.ctypes.data) == 0
    boxes = raw[:, :24].reshape(-1, 6, 4).astype(np.float64)
    codes = raw[:, 24:28].view(np.int32)
    for ni in range(info.nnodes4):
        p = q[ni, :3].view(np.float32).astype(np.float64)
        steps = q[ni, [3, 14, 15]].view(np.float32).astype(np.float64)
        for c in range(4):
            if int(codes[ni, c]) == np.iinfo(np.int32).min:
                continue
            for a in range(3):
                ql = (int(q[ni, 8 + 2 * a]) >> (8 * c)) & 0xFF
                qh = (int(q[ni, 9 + 2 * a]) >> (8 * c)) & 0xFF
                assert Fraction(p[a]) + ql * Fraction(steps[a]) <= Fraction(boxes[ni, 2 * a, c])
                assert Fraction(p[a]) + qh * Fraction(steps[a]) >= Fraction(boxes[ni, 2 * a + 1, c])
    L.pt_scene_free(h)


def test_bvh4_quantized_refused_for_huge_extents(L):
    """Extents that need steps above 2^60 (here ~1e25) make the quantized nodes unusable:
    the scene reports quant = 0 (the library then walks the float four-wide nodes)."""
    s = _shifted(scenes.tiny(), (0.0, 0.0, 0.0), scale=1.0e24)
    st, h, keep = _create(L, s)
    assert st == 0
    info, raw = _bvh4(L, h)
    assert info.quant == 0
    L.pt_scene_free(h)


def test_bvh4_empty_and_single_leaf(L):
    s = scenes.tiny()
    one = dict(s)
    one["tris"] = np.asarray(s["tris"])[:3]
    one["tri_mat"] = np.asarray(s["tri_mat"])[:3]
    for sc in (one,):
        st, h, keep = _create(L, scenes.Scene(sc))
        assert st == 0
        info, raw = _bvh4(L, h)
        codes = raw[:, 24:28].view(np.int32)
        assert info.nnodes4 == 1 and codes[0, 0] < 0 and (codes[0, 1:] == np.iinfo(np.int32).min).all()
        L.pt_scene_free(h)


@pytest.mark.parametrize("ntri,seed", [(24, 1), (36, 2), (40, 3)])
def test_bvh4_collapse_is_optimal(L, ntri, seed):
    """The four-wide collapse chooses which binary nodes root four-wide nodes so that their
    summed surface area (the visit cost; leaves cost the same wherever they land) is least:
    checked against every valid choice on small random trees (brute force)."""
    import itertools

    s = dict(scenes.furnace())
    rng = np.random.default_rng(seed)
    cen = rng.uniform(0.0, 10.0, (ntri, 1, 3))
    cen[: ntri // 2] *= 0.3                                   # a cluster and a spread
    s["tris"] = (cen + rng.uniform(-0.4, 0.4, (ntri, 3, 3))).astype(np.float32)
    s["tri_mat"] = np.zeros(ntri, np.uint32)
    st, h, keep = _create(L, s)
    assert st == 0
    info = capi.SceneInfo()
    L.pt_scene_get_info(h, C.byref(info))
    n2 = np.zeros((info.nnodes, 16), np.float32)
    order = np.zeros(ntri, np.uint32)
    L.pt_scene_export_bvh(h, n2.ctypes.data, order.ctypes.data)
    _, raw = _bvh4(L, h)
    L.pt_scene_free(h)
    EMPTY = np.iinfo(np.int32).min
    codes2 = n2[:, 12:14].view(np.int32)

    def area(lo, hi):
        d = np.asarray(hi, np.float64) - np.asarray(lo, np.float64)
        return d[0] * d[1] + d[1] * d[2] + d[2] * d[0]

    def child_boxes(k):
        f = n2[k].astype(np.float64)
        return [((f[0], f[2], f[8]), (f[1], f[3], f[9])), ((f[4], f[6], f[10]), (f[5], f[7], f[11]))]

    def node_area(k):
        bs = [b for b, c in zip(child_boxes(k), codes2[k]) if c != EMPTY]
        lo = np.min([b[0] for b in bs], axis=0)
        hi = np.max([b[1] for b in bs], axis=0)
        return area(lo, hi)

    inner = [k for k in range(info.nnodes)]
    assert 4 <= len(inner) <= 18, len(inner)                # brute force stays small

    def entries(k, opened):
        n = 0
        for c in codes2[k]:
            if c == EMPTY:
                continue
            n += entries(int(c), opened) if (c >= 0 and int(c) in opened) else 1
        return n

    best = np.inf
    others = inner[1:]
    for r in range(len(others) + 1):
        for opened in itertools.combinations(others, r):
            op = set(opened)
            roots = [k for k in inner if k not in op]
            if all(entries(k, op) <= 4 for k in roots):
                best = min(best, sum(node_area(k) for k in roots))
    # cost of the exported four-wide tree: the root's box plus every inner entry's box
    boxes = raw[:, :24].reshape(-1, 6, 4).astype(np.float64)
    codes4 = raw[:, 24:28].view(np.int32)
    valid = codes4[0] != EMPTY
    lo0 = [boxes[0, 2 * a][valid].min() for a in range(3)]
    hi0 = [boxes[0, 2 * a + 1][valid].max() for a in range(3)]
    got = area(lo0, hi0)
    for n in range(len(raw)):
        for j in range(4):
            if codes4[n, j] >= 0:
                got += area([boxes[n, 0, j], boxes[n, 2, j], boxes[n, 4, j]], [boxes[n, 1, j], boxes[n, 3, j], boxes[n, 5, j]])
    assert got <= best * (1 + 1e-9), (got, best)
    assert got >= best * (1 - 1e-9), (got, best)
