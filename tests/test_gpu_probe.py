"""Gather-rate probe (sr_probe_gather): its checksum is the sum of the
gathered values, computed here with numpy, for masked and clamped ids and a
ragged last tile; its time is positive."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sr():
    import paper_1806_00762_amd as sr
    sr.lib()
    return sr


@pytest.fixture(scope="module")
def ctx(sr):
    c = sr.Context(0, 0)
    yield c
    c.close()


@pytest.mark.parametrize("m,n,mask", [(1, 1, 0xFFFFFFFF), (2047, 1000, 0xFFFFFFFF), (2049, 5000, 0x00FFFFFF),
                                      (1 << 20, 1 << 16, 0x00FFFFFF), (3 * 2048 + 5, 300, 0xFFFFFFFF)])
def test_probe_checksum(sr, ctx, m, n, mask):
    rng = np.random.default_rng(m + n)
    if mask == 0xFFFFFFFF:
        words = rng.integers(0, n + 50, size=m, dtype=np.int64).astype(np.uint32)  # ids past n are clamped
    else:
        words = rng.integers(0, 2 ** 32, size=m, dtype=np.uint64).astype(np.uint32)
    vals = rng.integers(0, 2 ** 32, size=n, dtype=np.uint64).astype(np.uint32)
    ids = np.minimum(words & np.uint32(mask), np.uint32(n - 1)).astype(np.int64)
    want = int(vals[ids].astype(np.uint64).sum(dtype=np.uint64))
    say(f"case probe m={m} n={n} mask={mask:#x}")
    ms, cs = sr.probe_gather(ctx, words, mask, vals, repeats=3)
    say(f"  {ms:.4f} ms")
    assert cs == want
    assert ms > 0
