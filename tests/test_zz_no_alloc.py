"""The ownership read-out that allocates nothing, against the one that does.

vlb_read_ownership_noalloc stages its results in the library's static
device array, in chunks of whole tiles; vlb_read_ownership allocates its
staging buffers per call.  Both run the same kernel, so the integer outputs
must be identical.  Two calls in a row, the second on a smaller domain (the
array then still holds the first call's larger contents): a dense cavity
read in several chunks (per-tile lists), then a small channel (scan form).
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vlb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_23802_amd import vlb as v
    v.lib()  # fails loudly if the HIP library is missing
    return v


def compare(vlb, dom):
    a = vlb.vlb_read_ownership(dom.h, dom.nx, dom.ny, dom.kmax)
    b = vlb.vlb_read_ownership_noalloc(dom.h, dom.nx, dom.ny, dom.kmax)
    for x, y in zip(a, b):
        assert x.shape == y.shape
        assert np.array_equal(x, y)
    return a


def test_noalloc_ownership_matches_allocating_read(vlb):
    # 1536 x 1536 cells, 2048 disks: 9216 tiles, read in 6 chunks (kmax 4)
    d, ps = W.c3_dense()
    print("case: noalloc ownership, dense cavity 1536^2, 2048 disks",
          flush=True)
    dom = vlb.Domain(d, ps, "fp32").init().step(3)
    cnt, _, full = compare(vlb, dom)
    assert int(cnt.sum()) > 2048 * 150 and int(full.sum()) > 0
    dom.close()
    # a smaller domain on the same GPU: 128 x 64 cells, one disk
    d, ps = W.c1_tiny()
    print("case: noalloc ownership, tiny channel 128x64", flush=True)
    dom = vlb.Domain(d, ps, "fp64").init().step(2)
    cnt, ids, _ = compare(vlb, dom)
    assert int(cnt.sum()) > 200 and int((ids >= 0).sum()) == int(cnt.sum())
    dom.close()
