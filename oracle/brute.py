"""Float64 brute-force closest hit (numpy), an external pin for the oracle.

TEST INFRASTRUCTURE ONLY.  Every ray is tested against every triangle with
the Moller-Trumbore formulation evaluated in float64, which is independent of
the oracle's float32 watertight test.  Returns the nearest (t, prim) with t > 0
and the second-nearest distinct-prim distance, both in float64.
"""
from __future__ import annotations

import numpy as np


def closest_hits(tris: np.ndarray, rays: np.ndarray, chunk: int = 256):
    tris = np.asarray(tris, np.float64).reshape(-1, 3, 3)
    rays = np.asarray(rays, np.float32).reshape(-1, 8)
    o = rays[:, 0:3].astype(np.float64)
    d = rays[:, 4:7].astype(np.float64)
    excl = rays[:, 3].view(np.int32)
    v0 = tris[:, 0]
    e1 = tris[:, 1] - v0
    e2 = tris[:, 2] - v0
    n = rays.shape[0]
    prim = np.full(n, -1, np.int64)
    t1 = np.full(n, np.inf)
    t2 = np.full(n, np.inf)
    idx = np.arange(tris.shape[0])
    for s in range(0, n, chunk):
        oo = o[s:s + chunk, None, :]
        dd = d[s:s + chunk, None, :]
        p = np.cross(dd, e2[None])
        det = np.einsum("rtk,tk->rt", p, e1)
        with np.errstate(divide="ignore", invalid="ignore"):
            inv = 1.0 / det
            tv = oo - v0[None]
            u = np.einsum("rtk,rtk->rt", tv, p) * inv
            q = np.cross(tv, e1[None])
            v = np.einsum("rtk,rtk->rt", dd, q) * inv
            t = np.einsum("tk,rtk->rt", e2, q) * inv
        ok = (det != 0) & (u >= 0) & (v >= 0) & (u + v <= 1) & (t > 0)
        ok &= idx[None, :] != excl[s:s + chunk, None]
        tt = np.where(ok, t, np.inf)
        order = np.argsort(tt, axis=1, kind="stable")[:, :2]
        r = np.arange(tt.shape[0])
        best = tt[r, order[:, 0]]
        sec = tt[r, order[:, 1]] if tt.shape[1] > 1 else np.full(tt.shape[0], np.inf)
        prim[s:s + chunk] = np.where(np.isfinite(best), order[:, 0], -1)
        t1[s:s + chunk] = best
        t2[s:s + chunk] = sec
    return prim, t1, t2
