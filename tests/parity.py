"""Comparison of a GPU render with the oracle's.

The bar: hit primitive ids bit-exact except on rays whose two nearest hits lie
within 1e-6 relative t (a pixel that diverges on such a ray, and in reuse mode
its whole tile, is excluded from its later bounces and from the image check,
and at most 1e-5 of the checked pixels may be excluded); hit distance within
1e-5 relative and image RMSE within 1e-4.  Because both sides follow one
binary32 operation order without contraction, the comparison also asserts what
that order makes exact: every traced ray (origin, excluded primitive,
direction, pixel) bit for bit at every bounce, the hit distance bit for bit
wherever the ids agree, and the radiance bit for bit on every checked pixel."""
import numpy as np

TIE_REL = 1e-6
T_REL = 1e-5
RMSE = 1e-4
MAX_EXCLUDED = 1e-5


def _np(a):
    return a.cpu().numpy() if hasattr(a, "cpu") else np.asarray(a)


def compare_render(gpu: dict, orc: dict, tile=(8, 8), mode="incoherent", pixel_mask=None, check_rays=True):
    hp_g, ht_g, rad_g = _np(gpu["hit_prim"]), _np(gpu["hit_t"]), _np(gpu["radiance"])
    hp_o, ht_o, t2_o, rad_o = orc["hit_prim"], orc["hit_t"], orc["hit_t2"], orc["radiance"]
    if check_rays:
        assert "rays" in gpu and "rays" in orc, "render both sides with their traced rays"
        rays_g, rays_o = _np(gpu["rays"]).view(np.uint32), orc["rays"].view(np.uint32)
    B1, spp, h, w = hp_o.shape
    sel = np.ones((h, w), bool) if pixel_mask is None else pixel_mask
    excluded = np.zeros((spp, h, w), bool)
    ties = 0
    rays_checked = 0
    for b in range(B1):
        live = sel[None] & ~excluded
        if check_rays:
            diff = (rays_g[b] != rays_o[b]).any(axis=-1) & live
            assert not diff.any(), (f"bounce {b}: {int(diff.sum())} traced rays differ, e.g. at "
                                    f"{np.argwhere(diff)[:3].tolist()}")
            rays_checked += int((live & (hp_o[b] != -2)).sum())
        mism = (hp_g[b] != hp_o[b]) & live
        with np.errstate(invalid="ignore"):
            tie = (t2_o[b] - ht_o[b]) <= TIE_REL * ht_o[b]
        bad = mism & ~tie
        assert not bad.any(), (f"bounce {b}: {int(bad.sum())} prim mismatches, e.g. at "
                               f"{np.argwhere(bad)[:3].tolist()} gpu={hp_g[b][bad][:3]} oracle={hp_o[b][bad][:3]}")
        newly = mism & tie
        if newly.any():
            ties += int(newly.sum())
            if mode.startswith("reuse"):
                W, H = tile
                for s, y, x in np.argwhere(newly):
                    excluded[s, (y // H) * H:(y // H + 1) * H, (x // W) * W:(x // W + 1) * W] = True
            excluded |= newly
        keep = sel[None] & ~excluded & (hp_o[b] == hp_g[b])
        hit = keep & (hp_o[b] >= 0)
        if hit.any():
            rel = np.abs(ht_g[b][hit].astype(np.float64) - ht_o[b][hit]) / ht_o[b][hit]
            assert rel.max() <= T_REL, f"bounce {b}: t rel err {rel.max()}"
            same = ht_g[b][hit].view(np.uint32) == ht_o[b][hit].view(np.uint32)
            assert same.all(), f"bounce {b}: {int((~same).sum())} hit distances differ in their last bits"
        nohit = keep & (hp_o[b] < 0)
        assert np.all(np.isinf(ht_g[b][nohit])), f"bounce {b}: finite t on a miss"
    pix_ok = sel & ~excluded.any(axis=0)
    err = rad_g[pix_ok].astype(np.float64) - rad_o[pix_ok]
    rmse = float(np.sqrt(np.mean(err ** 2))) if err.size else 0.0
    assert rmse <= RMSE, f"radiance rmse {rmse}"
    n_excl = int(excluded.any(axis=0).sum())
    assert n_excl <= MAX_EXCLUDED * sel.sum(), f"too many excluded pixels: {n_excl} of {int(sel.sum())}"
    same_rad = rad_g[pix_ok].view(np.uint32) == rad_o[pix_ok].view(np.uint32)
    assert same_rad.all(), f"radiance differs in the last bits on {int((~same_rad).any(axis=-1).sum())} pixels"
    return dict(ties=ties, excluded=n_excl, rays_checked=rays_checked, pixels=int(pix_ok.sum()), rmse=rmse)
