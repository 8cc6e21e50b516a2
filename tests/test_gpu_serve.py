"""Batched serving through the C ABI: every result is identical alone and in
the mix, and identical to the oracle's least model."""
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


def _make_input(req):
    return dev(dlgen.to_dense(req.n, dlgen.request_edges(req)))


def _alone(dl, req):
    a = _make_input(req)
    if req.kind == "tc":
        return dl.dl_tc(a, method=dl.DL_TC_SQUARE, prec="i8")
    return dl.dl_sg(a, prec="i8")


def _oracle(req):
    a = dlgen.to_dense(req.n, dlgen.request_edges(req))
    return oracle.tc_seminaive(a)[0] if req.kind == "tc" else oracle.sg_seminaive(a)[0]


def test_mixed_stream_alone_vs_mix(dl):
    from paper_1608_00139_amd.serve import run_stream

    reqs = dlgen.serving_stream(40, seed=5, rate=0.0, n_lo=64, n_hi=700)
    # pool for about a third of the stream: forces waits and continuous admission
    pool = sum(5 * ((r.n + 63) // 64 * 64) ** 2 for r in reqs) // 3
    announce("serve mix", len(reqs), pool)
    stats, results = run_stream(reqs, _make_input, pool_bytes=pool, max_active=64, keep_results=True)
    assert len(stats.completions) == len(reqs)
    assert stats.eagain > 0
    for r in reqs:
        got, iters = results[r.rid]
        alone, it_alone = _alone(dl, r)
        assert np.array_equal(host(got), host(alone)), (r.rid, r.kind, r.n)
        assert iters == it_alone, (r.rid, iters, it_alone)
        assert np.array_equal(host(got), _oracle(r)), (r.rid, r.kind, r.n)


def test_submit_between_rounds(dl):
    reqs = dlgen.serving_stream(12, seed=9, rate=0.0, n_lo=64, n_hi=400)
    b = dl.Batch(pool_bytes=1 << 28, max_active=16)
    done = {}
    queue = list(reqs)
    announce("serve interleaved")
    rounds = 0
    while queue or len(done) < len(reqs):
        if queue and rounds % 2 == 0:  # two new requests every other round
            for r in queue[:2]:
                slot = b.dl_batch_submit(b.TC if r.kind == "tc" else b.SG, _make_input(r), r.rid)
                assert slot is not None
            queue = queue[2:]
        b.dl_batch_step()
        rounds += 1
        for tag, slot, iters in b.dl_batch_poll():
            r = reqs[tag]
            out = dev(np.zeros((r.n, r.n), np.uint8))
            ones = b.dl_batch_fetch(slot, out)
            assert ones == int(host(out).sum())
            done[tag] = (host(out), iters)
        assert rounds < 400
    for r in reqs:
        alone, it_alone = _alone(dl, r)
        assert np.array_equal(done[r.rid][0], host(alone)) and done[r.rid][1] == it_alone


def test_edge_requests(dl):
    b = dl.Batch(pool_bytes=1 << 24, max_active=4)
    announce("serve edge cases")
    empty = dev(np.zeros((70, 70), np.uint8))
    one = dev(np.zeros((1, 1), np.uint8))
    s0 = b.dl_batch_submit(b.TC, empty, 0)
    s1 = b.dl_batch_submit(b.SG, one, 1)
    s2 = b.dl_batch_submit(b.TC, dev(np.ones((3, 3), np.uint8)), 2)
    got = {}
    for _ in range(20):
        b.dl_batch_step()
        for tag, slot, iters in b.dl_batch_poll():
            n = {0: 70, 1: 1, 2: 3}[tag]
            out = dev(np.zeros((n, n), np.uint8))
            b.dl_batch_fetch(slot, out)
            got[tag] = (host(out), iters)
        if len(got) == 3:
            break
    assert got[0][1] == 1 and got[0][0].sum() == 0
    assert got[1][1] == 2 and got[1][0].tolist() == [[1]]
    assert got[2][1] == 2 and got[2][0].all()  # every pair at distance 1: D = 1
    # a request larger than the pool is refused with DL_EAGAIN
    small = dl.Batch(pool_bytes=1 << 16, max_active=2)
    assert small.dl_batch_submit(small.TC, dev(np.zeros((300, 300), np.uint8)), 7) is None
    with pytest.raises(dl.DLError):
        b.dl_batch_fetch(3)  # never used slot
