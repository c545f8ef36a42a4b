"""Comparison of a GPU render with the oracle's, with the spec bar:
hit primitive ids bit-exact except on rays whose two nearest hits lie within
1e-6 relative t (a pixel that diverges on such a ray, and in reuse mode its
whole tile, is excluded from its later bounces and from the image check),
hit distance within 1e-5 relative, image RMSE within 1e-4."""
import numpy as np

TIE_REL = 1e-6
T_REL = 1e-5
RMSE = 1e-4


def compare_render(gpu: dict, orc: dict, tile=(8, 8), mode="incoherent", pixel_mask=None):
    hp_g = gpu["hit_prim"].cpu().numpy() if hasattr(gpu["hit_prim"], "cpu") else gpu["hit_prim"]
    ht_g = gpu["hit_t"].cpu().numpy() if hasattr(gpu["hit_t"], "cpu") else gpu["hit_t"]
    rad_g = gpu["radiance"].cpu().numpy() if hasattr(gpu["radiance"], "cpu") else gpu["radiance"]
    hp_o, ht_o, t2_o, rad_o = orc["hit_prim"], orc["hit_t"], orc["hit_t2"], orc["radiance"]
    B1, spp, h, w = hp_o.shape
    sel = np.ones((h, w), bool) if pixel_mask is None else pixel_mask
    excluded = np.zeros((spp, h, w), bool)
    ties = 0
    exact_t = True
    for b in range(B1):
        live = sel[None] & ~excluded
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
            exact_t &= bool(np.array_equal(ht_g[b][hit].view(np.uint32), ht_o[b][hit].view(np.uint32)))
        nohit = keep & (hp_o[b] < 0)
        assert np.all(np.isinf(ht_g[b][nohit])), f"bounce {b}: finite t on a miss"
    pix_ok = sel & ~excluded.any(axis=0)
    err = rad_g[pix_ok].astype(np.float64) - rad_o[pix_ok]
    rmse = float(np.sqrt(np.mean(err ** 2))) if err.size else 0.0
    assert rmse <= RMSE, f"radiance rmse {rmse}"
    assert excluded.any(axis=0).sum() <= max(1e-5 * sel.sum(), 16), f"too many excluded pixels {excluded.sum()}"
    exact_rad = bool(np.array_equal(rad_g[pix_ok].view(np.uint32), rad_o[pix_ok].view(np.uint32)))
    return dict(ties=ties, exact_t=exact_t, exact_radiance=exact_rad, rmse=rmse)
