"""The memory-level probe on the GPU: the cycle it writes through the buffer's
128-byte lines and the end point of the dependent-load chase are checked exactly on
the host; bandwidth and latency are positive and below the published HBM peak for a
buffer far larger than every cache."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_07182_amd import api
    return torch, api


def _cycle_end(nlines, steps, a=1664525 * 4 + 1, c=1013904223):
    i = 0
    for _ in range(steps):
        i = ((a * i + c) & 0xFFFFFFFF) & (nlines - 1)
    return i


@pytest.mark.parametrize("nbytes,steps", [(64 << 10, 777), ((1 << 20) + 4096, 5000), (24 << 20, 20000)])
def test_probe_cycle_and_chase_exact(env, nbytes, steps):
    torch, api = env
    buf = torch.zeros(nbytes, dtype=torch.uint8, device="cuda:0")
    _say(f"[gpu] probe {nbytes} B, {steps} steps")
    r = api.probe_memory(nbytes, 2, steps, buf)
    torch.cuda.synchronize()
    words = buf.view(torch.int32).cpu().numpy().view(np.uint32)
    nlines = 1 << int(np.floor(np.log2(nbytes // 128)))
    first = words[: nlines * 32].reshape(nlines, 32)[:, 0]
    i = np.arange(nlines, dtype=np.uint64)
    want = ((np.uint64(1664525 * 4 + 1) * i + np.uint64(1013904223)) & np.uint64(0xFFFFFFFF)) & np.uint64(nlines - 1)
    assert np.array_equal(first.astype(np.uint64), want)
    # a single cycle through every line
    seen = np.zeros(nlines, bool)
    j = 0
    for _ in range(nlines):
        assert not seen[j]
        seen[j] = True
        j = int(want[j])
    assert j == 0 and seen.all()
    assert int(words[2]) == _cycle_end(nlines, steps)
    assert r["read_gbps"] > 0 and r["chase_ns"] > 0


def test_probe_hbm_rate_below_peak(env):
    torch, api = env
    _say("[gpu] probe 2 GiB")
    r = api.probe_memory(2 << 30, 2, 2000)
    assert 500.0 < r["read_gbps"] < 8000.0 * 1.05
    assert r["chase_ns"] > 50.0
