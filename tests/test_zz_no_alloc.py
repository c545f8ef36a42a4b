"""pt_trace_static (the traversal without a workspace, its scratch a fixed array inside the
library) against pt_trace, both through the C ABI, on the same seeded rays: bit-exact hit
ids and distances, on two calls in a row (the second smaller, so it runs over the first
call's scratch contents), and against the oracle's closest hits."""
import sys

import numpy as np
import pytest

from paper_2310_07182_amd import scenes

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _rays(orc, s, n, seed):
    rng = np.random.default_rng(seed)
    tris = s["tris"].astype(np.float64)
    lo, hi = tris.reshape(-1, 3).min(0), tris.reshape(-1, 3).max(0)
    o = rng.uniform(lo, hi, (n, 3)).astype(np.float32)
    d = rng.normal(size=(n, 3))
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    ex = rng.integers(-1, len(tris), n).astype(np.int32)
    return orc.pack_rays(o, d, ex)


def test_trace_static_matches_trace(orc, torch_dev):
    from paper_2310_07182_amd import api
    s = scenes.mixed_small()
    sc = api.Scene(s)
    osc = orc.OracleScene(s)
    assert api.lib().pt_trace_static_scratch_bytes() <= 40 << 20
    for call, (n, seed, refill, wpc) in enumerate([(40009, 31, 0, 0), (7001, 32, 48, 4)]):
        rays = _rays(orc, s, n, seed)
        dr = torch_dev.from_numpy(rays).cuda()
        _say(f"[gpu] pt_trace_static call {call}: mixed_small n={n} refill={refill} waves_per_cu={wpc}")
        ps, ts = api.trace_static(sc, dr, refill, wpc)
        _say(f"[gpu] pt_trace call {call}: mixed_small n={n} refill={refill}")
        pw, tw = api.trace(sc, dr, refill)
        torch_dev.cuda.synchronize()
        ps, ts, pw, tw = ps.cpu().numpy(), ts.cpu().numpy(), pw.cpu().numpy(), tw.cpu().numpy()
        assert np.array_equal(ps, pw)
        assert np.array_equal(ts.view(np.uint32), tw.view(np.uint32))
        po, to, t2 = osc.trace(rays)
        with np.errstate(invalid="ignore"):
            tie = (t2 - to) <= 1e-6 * to
        assert np.all((ps == po) | tie)
        same = ps == po
        assert np.array_equal(ts[same].view(np.uint32), to[same].view(np.uint32))
        assert (po >= 0).sum() > n // 4


def test_trace_static_rejects_grid_beyond_scratch(torch_dev):
    from paper_2310_07182_amd import api
    from paper_2310_07182_amd.capi import PT_EINVAL, PtError
    sc = api.Scene(scenes.tiny())
    dr = torch_dev.zeros((64, 8), dtype=torch_dev.float32, device="cuda")
    cus = torch_dev.cuda.get_device_properties(0).multi_processor_count
    too_many = 2048 // cus + 1
    _say(f"[gpu] pt_trace_static waves_per_cu={too_many} on {cus} CUs (refused before any launch)")
    with pytest.raises(PtError) as ei:
        api.trace_static(sc, dr, 0, too_many)
    assert ei.value.status == PT_EINVAL and "static scratch" in str(ei.value)
    with pytest.raises(PtError):
        api.trace_static(sc, dr, 0, 33)
    # n = 0 does nothing and succeeds
    prim, t = api.trace_static(sc, dr[:0])
    assert prim.numel() == 0
