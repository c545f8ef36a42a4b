"""Seeded synthetic scenes: the shared input generator.

This module only produces inputs (triangles, per-triangle material ids, a
material table, an environment radiance and a camera).  It holds none of the
path tracer's arithmetic: no ray generation, intersection, sampling or
grouping.  Both the GPU library and the CPU oracle consume its output; the
oracle never imports the GPU path and vice versa.

The paper evaluates on five archived scenes (Breakfast, Salle de Bain, Living
room, Sibenik, Vokselia; Section 5) that are not available here.  These
procedural scenes stand in for them with the same character: a dense indoor
room of instanced meshes (~1M triangles, the 0.6M-1.9M range of Table 1) and a
large outdoor landscape (terrain plus trees), plus a tiny room for parity.

Material record (32 bytes, little endian), identical in every consumer:
    uint32 kind      0 = Lambertian (diffuse), 1 = GGX (glossy), 2 = mirror (specular)
    float  albedo[3] Lambert albedo / GGX Schlick F0 / mirror tint
    float  alpha     GGX roughness (alpha = roughness), unused otherwise
    float  emission[3]
Triangles are float32 [n][3][3] (vertex, xyz).
"""
from __future__ import annotations

import numpy as np

MATERIAL_DTYPE = np.dtype([("kind", "<u4"), ("albedo", "<f4", (3,)),
                           ("alpha", "<f4"), ("emission", "<f4", (3,))])
assert MATERIAL_DTYPE.itemsize == 32

LAMBERT, GGX, MIRROR = 0, 1, 2
BASE_SEED = 2310071820


# --------------------------------------------------------------------------
# base meshes (float64 vertices, int faces)
# --------------------------------------------------------------------------
def icosphere(level: int):
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t),
         (0, -1, -t), (0, 1, -t), (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9),
         (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2),
         (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10),
         (8, 6, 7), (9, 8, 1)]
    verts = np.array(v, dtype=np.float64)
    verts /= np.linalg.norm(verts, axis=1, keepdims=True)
    faces = np.array(f, dtype=np.int64)
    for _ in range(level):
        a, b, c = faces[:, 0], faces[:, 1], faces[:, 2]
        edges = np.concatenate([np.stack([a, b], 1), np.stack([b, c], 1), np.stack([c, a], 1)])
        key = np.sort(edges, axis=1)
        uniq, inv = np.unique(key, axis=0, return_inverse=True)
        inv = inv.reshape(-1)
        mid = verts[uniq[:, 0]] + verts[uniq[:, 1]]
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
        base = len(verts)
        verts = np.concatenate([verts, mid])
        nf = len(faces)
        ab, bc, ca = inv[:nf] + base, inv[nf:2 * nf] + base, inv[2 * nf:] + base
        faces = np.concatenate([np.stack([a, ab, ca], 1), np.stack([b, bc, ab], 1),
                                np.stack([c, ca, bc], 1), np.stack([ab, bc, ca], 1)])
    return verts, faces


def torus(R: float, r: float, nu: int, nv: int):
    u = np.arange(nu) * (2 * np.pi / nu)
    v = np.arange(nv) * (2 * np.pi / nv)
    uu, vv = np.meshgrid(u, v, indexing="ij")
    x = (R + r * np.cos(vv)) * np.cos(uu)
    y = r * np.sin(vv)
    z = (R + r * np.cos(vv)) * np.sin(uu)
    verts = np.stack([x, y, z], -1).reshape(-1, 3)
    i, j = np.meshgrid(np.arange(nu), np.arange(nv), indexing="ij")
    i2, j2 = (i + 1) % nu, (j + 1) % nv
    a, b, c, d = i * nv + j, i2 * nv + j, i2 * nv + j2, i * nv + j2
    faces = np.concatenate([np.stack([a, b, c], -1).reshape(-1, 3),
                            np.stack([a, c, d], -1).reshape(-1, 3)])
    return verts, faces


def rounded_box(n: int, half: float = 0.7, radius: float = 0.3):
    """Cube with n x n quads per face, pushed out to a rounded box."""
    g = np.linspace(-1.0, 1.0, n + 1)
    faces_v, faces_f = [], []
    base = 0
    for axis in range(3):
        for sign in (-1.0, 1.0):
            uu, vv = np.meshgrid(g, g, indexing="ij")
            p = np.zeros(uu.shape + (3,))
            p[..., axis] = sign
            p[..., (axis + 1) % 3] = uu
            p[..., (axis + 2) % 3] = vv
            if sign < 0:
                p = p[:, ::-1]
            faces_v.append(p.reshape(-1, 3))
            i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
            a = base + i * (n + 1) + j
            b = a + (n + 1)
            c = b + 1
            d = a + 1
            faces_f.append(np.concatenate([np.stack([a, b, c], -1).reshape(-1, 3),
                                           np.stack([a, c, d], -1).reshape(-1, 3)]))
            base += (n + 1) * (n + 1)
    v = np.concatenate(faces_v)
    inner = np.clip(v * (half + radius), -half, half)
    off = v * (half + radius) - inner
    ln = np.linalg.norm(off, axis=1, keepdims=True)
    ln[ln == 0] = 1.0
    v = inner + radius * off / ln
    return v, np.concatenate(faces_f)


def displaced_icosphere(level: int, rng: np.random.Generator):
    v, f = icosphere(level)
    freq = rng.uniform(2.0, 6.0, size=(4, 3))
    phase = rng.uniform(0.0, 2 * np.pi, size=4)
    amp = rng.uniform(0.03, 0.08, size=4)
    r = 1.0 + np.sum(amp[None, :] * np.sin(v @ freq.T + phase[None, :]), axis=1)
    return v * r[:, None], f


def quad(p0, p1, p2, p3):
    """Two triangles of the planar quad p0 p1 p2 p3 (counter-clockwise)."""
    return [(p0, p1, p2), (p0, p2, p3)]


def tessellated_quad(p0, p1, p2, p3, cell: float = 1.0):
    """Planar parallelogram p0 p1 p2 p3 split into ~cell-sized quads (2 tris each)."""
    p0, p1, p3 = (np.asarray(p, np.float64) for p in (p0, p1, p3))
    nu = max(1, int(round(np.linalg.norm(p1 - p0) / cell)))
    nv = max(1, int(round(np.linalg.norm(p3 - p0) / cell)))
    u = np.arange(nu + 1) / nu
    v = np.arange(nv + 1) / nv
    g = p0[None, None] + u[:, None, None] * (p1 - p0)[None, None] + v[None, :, None] * (p3 - p0)[None, None]
    a, b = g[:-1, :-1], g[1:, :-1]
    c, d = g[1:, 1:], g[:-1, 1:]
    t = np.concatenate([np.stack([a, b, c], 2).reshape(-1, 3, 3), np.stack([a, c, d], 2).reshape(-1, 3, 3)])
    return t


def random_rotation(rng: np.random.Generator):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def _drop_degenerate(tris64: np.ndarray, mat: np.ndarray):
    e1 = tris64[:, 1] - tris64[:, 0]
    e2 = tris64[:, 2] - tris64[:, 0]
    area = np.linalg.norm(np.cross(e1, e2), axis=1)
    keep = area > 1e-9
    return tris64[keep], mat[keep]


class Scene(dict):
    """dict with keys tris, tri_mat, mats, env, camera, name."""

    @property
    def ntri(self) -> int:
        return int(self["tris"].shape[0])


def _finish(name, tri_list, mat_list, mats, env, camera) -> Scene:
    tris = np.concatenate(tri_list).astype(np.float64)
    mat = np.concatenate(mat_list).astype(np.uint32)
    tris, mat = _drop_degenerate(tris, mat)
    return Scene(name=name,
                 tris=np.ascontiguousarray(tris.astype(np.float32)),
                 tri_mat=np.ascontiguousarray(mat),
                 mats=np.array(mats, dtype=MATERIAL_DTYPE),
                 env=np.asarray(env, dtype=np.float32),
                 camera=camera)


def _mat(kind, albedo, alpha=0.0, emission=(0.0, 0.0, 0.0)):
    return (kind, tuple(float(a) for a in albedo), float(alpha), tuple(float(e) for e in emission))


def _mesh_tris(v, f, rot, scale, pos):
    vv = (v * scale) @ rot.T + pos
    return vv[f]


# --------------------------------------------------------------------------
# configurations
# --------------------------------------------------------------------------
def tiny(seed: int = BASE_SEED + 0, spheres: int = 8, level: int = 2) -> Scene:
    """Open-front 10 m box room (5 quads) plus random icospheres, all Lambertian."""
    rng = np.random.default_rng(seed)
    mats, tris, mid = [], [], []
    S = 10.0
    room = [
        quad((0, 0, 0), (S, 0, 0), (S, 0, S), (0, 0, S)),        # floor
        quad((0, S, 0), (0, S, S), (S, S, S), (S, S, 0)),        # ceiling
        quad((0, 0, 0), (0, 0, S), (0, S, S), (0, S, 0)),        # left
        quad((S, 0, 0), (S, S, 0), (S, S, S), (S, 0, S)),        # right
        quad((0, 0, 0), (0, S, 0), (S, S, 0), (S, 0, 0)),        # back
    ]
    for q in room:
        mats.append(_mat(LAMBERT, rng.uniform(0.2, 0.8, 3)))
        tris.append(np.array(q, dtype=np.float64))
        mid.append(np.full(2, len(mats) - 1))
    v, f = icosphere(level)
    for _ in range(spheres):
        r = rng.uniform(0.5, 1.5)
        c = rng.uniform(r, S - r, 3)
        mats.append(_mat(LAMBERT, rng.uniform(0.2, 0.8, 3)))
        tris.append(_mesh_tris(v, f, np.eye(3), r, c))
        mid.append(np.full(len(f), len(mats) - 1))
    cam = dict(pos=(5.0, 5.0, 19.0), look_at=(5.0, 5.0, 0.0), up=(0.0, 1.0, 0.0), vfov=50.0)
    return _finish("tiny", tris, mid, mats, (1.0, 1.0, 1.0), cam)


def _instanced_room(name, seed, n_inst, size=(20.0, 8.0, 20.0), env=(0.05, 0.05, 0.05),
                    mix=(0.6, 0.3, 0.1), mesh_p=(0.35, 0.30, 0.10, 0.25)) -> Scene:
    rng = np.random.default_rng(seed)
    X, Y, Z = size
    mats, tris, mid = [], [], []
    room = [
        ((0, 0, 0), (X, 0, 0), (X, 0, Z), (0, 0, Z)),
        ((0, Y, 0), (0, Y, Z), (X, Y, Z), (X, Y, 0)),
        ((0, 0, 0), (0, 0, Z), (0, Y, Z), (0, Y, 0)),
        ((X, 0, 0), (X, Y, 0), (X, Y, Z), (X, 0, Z)),
        ((0, 0, 0), (0, Y, 0), (X, Y, 0), (X, 0, 0)),
        ((0, 0, Z), (X, 0, Z), (X, Y, Z), (0, Y, Z)),
    ]
    for q in room:
        mats.append(_mat(LAMBERT, rng.uniform(0.5, 0.8, 3)))
        t = tessellated_quad(*q, cell=1.0)
        tris.append(t)
        mid.append(np.full(len(t), len(mats) - 1))
    # four emissive ceiling panels: black Lambertian with emission 20
    mats.append(_mat(LAMBERT, (0, 0, 0), 0.0, (20.0, 20.0, 20.0)))
    e_id = len(mats) - 1
    yl = Y - 0.01
    for cx in (X * 0.3, X * 0.7):
        for cz in (Z * 0.3, Z * 0.7):
            q = quad((cx - 1, yl, cz - 1), (cx - 1, yl, cz + 1), (cx + 1, yl, cz + 1), (cx + 1, yl, cz - 1))
            tris.append(np.array(q, dtype=np.float64))
            mid.append(np.full(2, e_id))
    bases = [icosphere(3), torus(1.0, 0.35, 48, 24), None, rounded_box(11)]
    for _ in range(n_inst):
        m = rng.choice(4, p=mesh_p)
        if m == 2:
            v, f = displaced_icosphere(4, rng)
        else:
            v, f = bases[m]
        kind = rng.choice(3, p=mix)
        if kind == LAMBERT:
            mats.append(_mat(LAMBERT, rng.uniform(0.2, 0.8, 3)))
        elif kind == GGX:
            mats.append(_mat(GGX, rng.uniform(0.5, 0.95, 3), rng.uniform(0.05, 0.5)))
        else:
            mats.append(_mat(MIRROR, rng.uniform(0.7, 0.95, 3)))
        scale = rng.uniform(0.3, 0.9)
        pos = np.array([rng.uniform(1, X - 1), rng.uniform(0.4, Y - 2.0), rng.uniform(1, Z - 1)])
        tris.append(_mesh_tris(v, f, random_rotation(rng), scale, pos))
        mid.append(np.full(len(f), len(mats) - 1))
    cam = dict(pos=(X * 0.5, 1.7, Z - 0.5), look_at=(X * 0.5, 1.4, 0.0), up=(0.0, 1.0, 0.0), vfov=60.0)
    return _finish(name, tris, mid, mats, env, cam)


def indoor(seed: int = BASE_SEED + 1) -> Scene:
    """Closed 20x8x20 m room, 4 emissive ceiling panels, 500 random instances (~1.0M tris)."""
    return _instanced_room("indoor", seed, 500)


def mid(seed: int = BASE_SEED + 4) -> Scene:
    """50-instance room, ~100k triangles."""
    return _instanced_room("mid", seed, 50)


def glossy_only(seed: int = BASE_SEED + 5, n_inst: int = 12) -> Scene:
    """Small room where every surface is GGX or mirror (reuse must equal incoherent)."""
    s = _instanced_room("glossy_only", seed, n_inst, size=(10.0, 6.0, 10.0), env=(1.0, 1.0, 1.0),
                        mix=(0.0, 0.7, 0.3), mesh_p=(0.6, 0.4, 0.0, 0.0))
    mats = s["mats"].copy()
    for i in range(len(mats)):
        if mats[i]["kind"] == LAMBERT and np.any(mats[i]["albedo"] > 0):
            mats[i]["kind"] = GGX
            mats[i]["alpha"] = 0.3
    # the ceiling panels become black mirrors with emission
    for i in range(len(mats)):
        if np.all(mats[i]["albedo"] == 0):
            mats[i]["kind"] = MIRROR
    s["mats"] = mats
    return s


def furnace(rho: float = 0.5, emission: float = 1.0) -> Scene:
    """Closed 6-quad box, every face Lambertian albedo rho with emission E.

    Every path returns E * sum_{k=0..B} rho^k regardless of direction."""
    S = 4.0
    mats = [_mat(LAMBERT, (rho, rho, rho), 0.0, (emission, emission, emission))]
    room = [
        quad((0, 0, 0), (S, 0, 0), (S, 0, S), (0, 0, S)),
        quad((0, S, 0), (0, S, S), (S, S, S), (S, S, 0)),
        quad((0, 0, 0), (0, 0, S), (0, S, S), (0, S, 0)),
        quad((S, 0, 0), (S, S, 0), (S, S, S), (S, 0, S)),
        quad((0, 0, 0), (0, S, 0), (S, S, 0), (S, 0, 0)),
        quad((0, 0, S), (S, 0, S), (S, S, S), (0, S, S)),
    ]
    tris = [np.array(q, dtype=np.float64) for q in room]
    mid = [np.zeros(2, dtype=np.int64) for _ in room]
    cam = dict(pos=(2.0, 2.0, 2.0), look_at=(2.0, 2.0, 0.0), up=(0.0, 1.0, 0.0), vfov=90.0)
    return _finish("furnace", tris, mid, mats, (0.0, 0.0, 0.0), cam)


def mixed_small(seed: int = BASE_SEED + 6) -> Scene:
    """Small room with the indoor material mix (hybrid groups occur)."""
    return _instanced_room("mixed_small", seed, 16, size=(10.0, 6.0, 10.0), env=(0.2, 0.2, 0.2),
                           mesh_p=(0.6, 0.4, 0.0, 0.0))


# --------------------------------------------------------------------------
# landscape: fBm heightfield + scattered trees
# --------------------------------------------------------------------------
def _hash2(ix, iy, salt):
    h = (ix.astype(np.uint64) * np.uint64(0x9E3779B97F4A7C15)) ^ (iy.astype(np.uint64) * np.uint64(0xC2B2AE3D27D4EB4F)) ^ np.uint64(salt)
    h ^= h >> np.uint64(29)
    h *= np.uint64(0xBF58476D1CE4E5B9)
    h ^= h >> np.uint64(32)
    return (h >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def _value_noise(x, y, salt):
    ix = np.floor(x)
    iy = np.floor(y)
    fx = x - ix
    fy = y - iy
    ix = ix.astype(np.int64)
    iy = iy.astype(np.int64)
    sx = fx * fx * (3 - 2 * fx)
    sy = fy * fy * (3 - 2 * fy)
    n00 = _hash2(ix, iy, salt)
    n10 = _hash2(ix + 1, iy, salt)
    n01 = _hash2(ix, iy + 1, salt)
    n11 = _hash2(ix + 1, iy + 1, salt)
    return (n00 * (1 - sx) + n10 * sx) * (1 - sy) + (n01 * (1 - sx) + n11 * sx) * sy


def _value_noise_grid(x, y, salt):
    """_value_noise over the grid x[i] (first axis) by y[j] (second axis): the lattice
    values are hashed once and gathered, the same arithmetic per point."""
    ix = np.floor(x)
    iy = np.floor(y)
    fx = (x - ix)[:, None]
    fy = (y - iy)[None, :]
    ix = ix.astype(np.int64)
    iy = iy.astype(np.int64)
    sx = fx * fx * (3 - 2 * fx)
    sy = fy * fy * (3 - 2 * fy)
    lx = np.arange(ix.min(), ix.max() + 2, dtype=np.int64)
    ly = np.arange(iy.min(), iy.max() + 2, dtype=np.int64)
    G = _hash2(lx[:, None] + 0 * ly[None, :], ly[None, :] + 0 * lx[:, None], salt)
    gi = ix - lx[0]
    gj = iy - ly[0]
    rows0, rows1 = G[gi], G[gi + 1]
    n00, n01 = rows0[:, gj], rows0[:, gj + 1]
    n10, n11 = rows1[:, gj], rows1[:, gj + 1]
    return (n00 * (1 - sx) + n10 * sx) * (1 - sy) + (n01 * (1 - sx) + n11 * sx) * sy


def fbm_heightfield(n: int, seed: int, octaves: int = 8, amplitude: float = 300.0,
                    base_period: float = 1024.0) -> np.ndarray:
    """n x n heights (float64), value-noise fBm, lacunarity 2, gain 0.5."""
    rng = np.random.default_rng(seed)
    salts = rng.integers(0, 2 ** 62, size=octaves)
    xs = np.arange(n, dtype=np.float64)
    hgt = np.zeros((n, n), dtype=np.float64)
    amp, freq, norm = 1.0, 1.0 / base_period, 0.0
    for o in range(octaves):
        hgt += amp * (_value_noise_grid(xs * freq, xs * freq, int(salts[o])) - 0.5)
        norm += amp
        amp *= 0.5
        freq *= 2.0
    return hgt * (amplitude / norm)


def landscape(seed: int = BASE_SEED + 2, grid: int = 4096, trees: int = 20000,
              spacing: float = 1.0) -> Scene:
    """fBm terrain (2*(grid-1)^2 tris) plus scattered trees (~1.5k tris each)."""
    rng = np.random.default_rng(seed)
    hgt = fbm_heightfield(grid, seed)
    mats = [_mat(LAMBERT, (0.35, 0.30, 0.22)),              # terrain
            _mat(GGX, (0.6, 0.6, 0.6), 0.3),                 # wet rock patches
            _mat(LAMBERT, (0.30, 0.20, 0.12)),              # trunk
            _mat(LAMBERT, (0.15, 0.45, 0.12)),              # canopy
            _mat(GGX, (0.5, 0.7, 0.5), 0.2)]                 # glossy canopy
    g = grid
    xs = np.arange(g, dtype=np.float64) * spacing
    # vertices (i, j) -> (x = i*spacing, y = h, z = j*spacing)
    V = np.empty((g, g, 3), dtype=np.float32)
    V[..., 0] = xs[:, None]
    V[..., 2] = xs[None, :]
    V[..., 1] = hgt
    i = np.arange(g - 1)
    a = V[:-1, :-1]
    b = V[1:, :-1]
    c = V[1:, 1:]
    d = V[:-1, 1:]
    terrain = np.empty((2, g - 1, g - 1, 3, 3), dtype=np.float32)
    terrain[0, :, :, 0] = a
    terrain[0, :, :, 1] = d
    terrain[0, :, :, 2] = c
    terrain[1, :, :, 0] = a
    terrain[1, :, :, 1] = c
    terrain[1, :, :, 2] = b
    terrain = terrain.reshape(-1, 3, 3)
    del a, b, c, d, i
    # 20% of terrain patches glossy (by coarse cell)
    cell = (np.arange(g - 1) // 64)
    ci, cj = np.meshgrid(cell, cell, indexing="ij")
    gl = _hash2(ci, cj, 77) < 0.2
    tmat = np.where(np.broadcast_to(gl, (2, g - 1, g - 1)).reshape(-1), 1, 0).astype(np.uint32)
    # trees
    trunk_v, trunk_f = _cylinder(16, 7)
    canopy_v, canopy_f = icosphere(3)      # 1280 tris
    tree_tris, tree_mat = [], []
    ext = (g - 1) * spacing
    tx = rng.uniform(0.02 * ext, 0.98 * ext, trees)
    tz = rng.uniform(0.02 * ext, 0.98 * ext, trees)
    ii = np.clip((tx / spacing).astype(np.int64), 0, g - 1)
    jj = np.clip((tz / spacing).astype(np.int64), 0, g - 1)
    ty = hgt[ii, jj] - 0.3
    # batch all trees: trunk (224 tris) + one displaced canopy icosphere (1280) => 1504 tris
    H = rng.uniform(4.0, 10.0, trees)
    Rt = rng.uniform(0.15, 0.35, trees)
    Rc = rng.uniform(1.5, 3.5, trees)
    glossy = rng.uniform(size=trees) < 0.2
    base = np.stack([tx, ty, tz], 1)
    # trunk
    tv = trunk_v[None, :, :] * np.stack([Rt, H, Rt], 1)[:, None, :] + base[:, None, :]
    tree_tris.append(tv[:, trunk_f].reshape(-1, 3, 3).astype(np.float32))
    tree_mat.append(np.full(trees * len(trunk_f), 2, dtype=np.uint32))
    # canopy: icosphere squashed + per-tree wobble
    wob = rng.uniform(0.0, 2 * np.pi, (trees, 3))
    cv = canopy_v[None, :, :]
    r = 1.0 + 0.12 * np.sin(3.0 * cv[..., 0] + wob[:, None, 0:1][..., 0]) * np.cos(2.0 * cv[..., 2] + wob[:, None, 1:2][..., 0])
    cvv = cv * r[..., None] * np.stack([Rc, Rc * 1.3, Rc], 1)[:, None, :] + (base + np.stack([0 * H, H + Rc * 0.8, 0 * H], 1))[:, None, :]
    tree_tris.append(cvv[:, canopy_f].reshape(-1, 3, 3).astype(np.float32))
    tree_mat.append(np.repeat(np.where(glossy, 4, 3).astype(np.uint32), len(canopy_f)))
    tris = np.concatenate([terrain] + tree_tris)
    del terrain
    tri_mat = np.concatenate([tmat] + tree_mat)
    mid_x = 0.5 * ext
    cam_pos = np.array([mid_x, hgt[int(mid_x / spacing), int(0.1 * ext / spacing)] + 2.0, 0.1 * ext])
    pitch = np.deg2rad(-2.0)
    look = cam_pos + np.array([0.0, np.tan(pitch) * 100.0, 100.0])
    cam = dict(pos=tuple(cam_pos), look_at=tuple(look), up=(0.0, 1.0, 0.0), vfov=60.0)
    return Scene(name="landscape", tris=np.ascontiguousarray(tris), tri_mat=np.ascontiguousarray(tri_mat),
                 mats=np.array(mats, dtype=MATERIAL_DTYPE), env=np.array([1.0, 1.0, 1.0], np.float32),
                 camera=cam)


def _cylinder(n: int, rings: int):
    ang = np.arange(n) * (2 * np.pi / n)
    ys = np.linspace(0.0, 1.0, rings + 1)
    A, Yy = np.meshgrid(ang, ys, indexing="ij")
    v = np.stack([np.cos(A), Yy, np.sin(A)], -1).reshape(-1, 3)
    i, j = np.meshgrid(np.arange(n), np.arange(rings), indexing="ij")
    i2 = (i + 1) % n
    a = i * (rings + 1) + j
    b = i2 * (rings + 1) + j
    c = b + 1
    d = a + 1
    f = np.concatenate([np.stack([a, c, b], -1).reshape(-1, 3), np.stack([a, d, c], -1).reshape(-1, 3)])
    return v, f


CONFIGS = {
    "tiny": dict(scene=tiny, w=64, h=64, spp=1, bounces=2, tile=(4, 4), k=2),
    "indoor": dict(scene=indoor, w=1920, h=1080, spp=1, bounces=4, tile=(8, 8), k=8),
    "landscape": dict(scene=landscape, w=1920, h=1080, spp=1, bounces=3, tile=(8, 8), k=8),
    "mid": dict(scene=mid, w=512, h=512, spp=1, bounces=4, tile=(8, 8), k=8),
}
