"""dl_tc_noalloc: the plain closure for callers that cannot allocate, with
its buffers in a static device array, against dl_tc (and the oracle) on
consecutive calls that reuse that array, the second with a smaller input."""
from __future__ import annotations

import numpy as np
import pytest

import dlgen
import oracle
from tests.gpu_util import announce, dev, gpu, host

pytestmark = gpu


@pytest.fixture(scope="module")
def dl():
    import paper_1608_00139_amd as m

    m.load()
    return m


@pytest.mark.parametrize("prec", ["f32", "i8", "bf16", "fp8", "fp4"])
def test_noalloc_matches_dl_tc_on_consecutive_calls(dl, prec):
    import torch

    for n, seed in ((512, 1), (300, 2), (97, 3), (1, 4)):
        a = dlgen.to_dense(n, dlgen.er_edges(n, 2.0 / n if n > 1 else 0.0, seed, self_loops=True))
        announce("noalloc", prec, n)
        ref, _, it_ref, _ = oracle.tc_seminaive(a)
        want, it_want = dl.dl_tc(dev(a), method=dl.DL_TC_PLAIN, prec=prec)
        out = torch.full((n, n + 5), 7, dtype=torch.uint8, device="cuda")
        got, it = dl.dl_tc_noalloc(dev(a), prec=prec, out=out[:, :n])
        assert it == it_want == it_ref
        assert torch.equal(got, want)
        assert np.array_equal(host(got), ref)
        assert bool((out[:, n:] == 7).all())


def test_noalloc_limits_and_empty(dl):
    a = np.zeros((513, 513), np.uint8)
    with pytest.raises(dl.DLError) as ei:
        dl.dl_tc_noalloc(dev(a), prec="i8")
    assert ei.value.status == 1
    r, it = dl.dl_tc_noalloc(dev(np.zeros((40, 40), np.uint8)), prec="f32")
    assert it == 1 and not bool(r.any())
    cyc = np.roll(np.eye(512, dtype=np.uint8), 1, axis=1)  # D = 512: the longest series
    r, it = dl.dl_tc_noalloc(dev(cyc), prec="i8")
    assert it == 513 and bool(r.all())
