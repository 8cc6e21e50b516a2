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


@pytest.mark.parametrize("lookahead", [0, 1])
def test_mixed_stream_alone_vs_mix(dl, lookahead):
    from paper_1608_00139_amd.serve import run_stream

    reqs = dlgen.serving_stream(40, seed=5, rate=0.0, n_lo=64, n_hi=700)
    # pool for about a third of the stream: forces waits and continuous admission
    pool = sum(5 * ((r.n + 63) // 64 * 64) ** 2 for r in reqs) // 3
    announce("serve mix", len(reqs), pool, lookahead)
    stats, results = run_stream(reqs, _make_input, pool_bytes=pool, max_active=64, keep_results=True,
                                lookahead=lookahead)
    assert len(stats.completions) == len(reqs)
    assert stats.eagain > 0
    for r in reqs:
        got, iters = results[r.rid]
        alone, it_alone = _alone(dl, r)
        assert np.array_equal(host(got), host(alone)), (r.rid, r.kind, r.n)
        assert iters == it_alone, (r.rid, iters, it_alone)
        assert np.array_equal(host(got), _oracle(r)), (r.rid, r.kind, r.n)


@pytest.mark.parametrize("lookahead", [0, 1])
def test_submit_between_rounds(dl, lookahead):
    """Two new requests every other round into four slots, so finished slots
    are fetched and reused while (with look-ahead) a round is in flight."""
    reqs = dlgen.serving_stream(12, seed=9, rate=0.0, n_lo=64, n_hi=400)
    b = dl.Batch(pool_bytes=1 << 28, max_active=4, lookahead=lookahead)
    done = {}
    queue = list(reqs)
    announce("serve interleaved", lookahead)
    rounds = 0
    while queue or len(done) < len(reqs):
        if queue and rounds % 2 == 0:  # up to two new requests every other round
            for _ in range(2):
                if not queue:
                    break
                r = queue[0]
                slot = b.dl_batch_submit(b.TC if r.kind == "tc" else b.SG, _make_input(r), r.rid)
                if slot is None:
                    break
                queue = queue[1:]
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


@pytest.mark.parametrize("lookahead", [0, 1])
def test_fetch_before_poll(dl, lookahead):
    """A request fetched without being polled is not reported by a later
    poll, also after its slot has been reused by a new request."""
    b = dl.Batch(pool_bytes=1 << 24, max_active=2, lookahead=lookahead)
    announce("serve fetch before poll", lookahead)
    n_path = 256  # a directed path: about log2(n) + 2 squaring iterations
    path = np.zeros((n_path, n_path), np.uint8)
    path[np.arange(n_path - 1), np.arange(1, n_path)] = 1
    s_empty = b.dl_batch_submit(b.TC, dev(np.zeros((70, 70), np.uint8)), 10)
    s_path = b.dl_batch_submit(b.TC, dev(path), 11)
    for _ in range(3):  # the empty relation is finished after one or two rounds
        b.dl_batch_step()
    assert b.dl_batch_fetch(s_empty) == 0  # not polled
    three = np.ones((3, 3), np.uint8)
    s_new = b.dl_batch_submit(b.TC, dev(three), 12)
    assert s_new == s_empty  # the fetched slot is reused
    polled = {}
    for _ in range(30):
        b.dl_batch_step()
        for tag, slot, iters in b.dl_batch_poll():
            assert tag != 10, "a fetched request was polled"
            n = {11: n_path, 12: 3}[tag]
            out = dev(np.zeros((n, n), np.uint8))
            b.dl_batch_fetch(slot, out)
            polled[tag] = (host(out), iters)
        if len(polled) == 2:
            break
    assert sorted(polled) == [11, 12]
    assert np.array_equal(polled[11][0], oracle.tc_seminaive(path)[0])
    assert polled[12][0].all() and polled[12][1] == 2


@pytest.mark.parametrize("lookahead", [0, 1])
def test_edge_list_admission(dl, lookahead):
    """Requests admitted as device edge lists give the same models and
    iteration counts as dense admission and the oracle; repeated pairs count
    once, pairs outside [0, n) are skipped, an empty list is the empty relation."""
    import torch

    from paper_1608_00139_amd.serve import run_stream

    reqs = dlgen.serving_stream(30, seed=11, rate=0.0, n_lo=64, n_hi=900)

    def edges_of(r):
        e = dlgen.request_edges(r).astype(np.int32)
        rng = np.random.default_rng(r.rid)
        extra = [e[: min(len(e), 5)], np.array([[r.n, 0], [0, r.n], [-1, 3], [2, -5]], np.int32)]
        return torch.from_numpy(np.concatenate([e] + extra)).cuda()

    announce("serve edges", len(reqs), lookahead)
    stats, results = run_stream(reqs, edges_of, pool_bytes=1 << 30, max_active=16, keep_results=True,
                                lookahead=lookahead)
    _, dense = run_stream(reqs, _make_input, pool_bytes=1 << 30, max_active=16, keep_results=True)
    for r in reqs:
        got, iters = results[r.rid]
        assert np.array_equal(host(got), host(dense[r.rid][0])), (r.rid, r.kind, r.n)
        assert iters == dense[r.rid][1]
        assert np.array_equal(host(got), _oracle(r)), (r.rid, r.kind, r.n)
    # model sizes: ones[1] (the relation itself) counts distinct pairs
    b = dl.Batch(pool_bytes=1 << 26, max_active=4, lookahead=lookahead)
    n = 100
    e = np.array([[1, 2], [2, 3], [1, 2], [1, 2], [3, 1], [99, 0]], np.int32)
    slot = b.dl_batch_submit_edges(dl.Batch.TC, n, torch.from_numpy(e).cuda(), 7)
    empty = b.dl_batch_submit_edges(dl.Batch.TC, 5, torch.zeros((0, 2), dtype=torch.int32, device="cuda"), 8)
    fin = {}
    while len(fin) < 2:
        b.dl_batch_step()
        for tag, sl, iters in b.dl_batch_poll():
            out = torch.empty((n if tag == 7 else 5,) * 2, dtype=torch.uint8, device="cuda")
            ones = b.dl_batch_fetch(sl, out)
            fin[tag] = (host(out), iters, ones)
    a = np.zeros((n, n), np.uint8)
    a[e[:, 0], e[:, 1]] = 1
    ref, _, it, _ = oracle.tc_seminaive(a)
    assert np.array_equal(fin[7][0], ref) and fin[7][2] == int(ref.sum())
    assert fin[8][1] == 1 and fin[8][2] == 0 and not fin[8][0].any()
    b.close()


@pytest.mark.parametrize("lookahead", [0, 1])
def test_grouped_admission_many_small(dl, lookahead):
    """Forty edge-list requests admitted before one round (one grouped clear
    and scatter for all of them): sizes 1..90, empty lists, repeated and
    out-of-range pairs, lists that end inside a wave of the scatter; every
    model, count of distinct pairs and iteration count equals the oracle's."""
    import torch

    rng = np.random.default_rng(5)
    b = dl.Batch(pool_bytes=1 << 28, max_active=64, lookahead=lookahead)
    cases = {}
    for tag in range(40):
        n = int(rng.integers(1, 91))
        kind = dl.Batch.TC if tag % 3 else dl.Batch.SG
        m = 0 if tag % 7 == 0 else int(rng.integers(1, 3 * n + 2))
        if kind == dl.Batch.SG:
            par = dlgen.forest_parents(n, tag)
            e = np.stack([np.nonzero(par >= 0)[0], par[par >= 0]], axis=1).astype(np.int32)[: m]
        else:
            e = rng.integers(-2, n + 2, size=(m, 2)).astype(np.int32)
        a = np.zeros((n, n), np.uint8)
        ok = (e[:, 0] >= 0) & (e[:, 1] >= 0) & (e[:, 0] < n) & (e[:, 1] < n) if len(e) else np.zeros(0, bool)
        a[e[ok, 0], e[ok, 1]] = 1
        slot = b.dl_batch_submit_edges(kind, n, torch.from_numpy(e.reshape(-1, 2)).cuda(), tag)
        assert slot is not None
        cases[tag] = (kind, n, a)
    announce("serve grouped admission", len(cases), lookahead)
    fin = {}
    for _ in range(200):
        b.dl_batch_step()
        for tag, sl, iters in b.dl_batch_poll():
            n = cases[tag][1]
            out = torch.empty((n, n), dtype=torch.uint8, device="cuda")
            ones = b.dl_batch_fetch(sl, out)
            fin[tag] = (host(out), iters, ones)
        if len(fin) == len(cases):
            break
    assert len(fin) == len(cases)
    for tag, (kind, n, a) in cases.items():
        if kind == dl.Batch.TC:
            ref, _, _, _ = oracle.tc_seminaive(a)
            _, hist = oracle.bfs(a, want_matrix=False)
            it_ref = oracle.square_schedule_from_hist(hist)[0]
        else:
            ref, _, it_ref, _ = oracle.sg_seminaive(a)
        got, iters, ones = fin[tag]
        assert np.array_equal(got, ref), (tag, kind, n)
        assert iters == it_ref, (tag, kind, n)
        assert ones == int(ref.sum()), (tag, kind, n)
    b.close()


@pytest.mark.parametrize("tile", [64, 256])
def test_forced_tile_table(dl, tile):
    """Every request on one tile size (64 x 64 tiles for sizes up to 1500,
    or 256 x 256 tiles for requests of 60 constants) gives the oracle's model
    and the single-call iteration count."""
    import torch

    from paper_1608_00139_amd.serve import run_stream

    reqs = dlgen.serving_stream(16, seed=31, rate=0.0, n_lo=60, n_hi=1500)

    def edges_of(r):
        return torch.from_numpy(dlgen.request_edges(r).astype(np.int32)).cuda()

    announce("serve forced tiles", tile)
    stats, results = run_stream(reqs, edges_of, pool_bytes=1 << 31, max_active=16, keep_results=True,
                                lookahead=1, tiles=[{"n": 16384, "tile": tile}])
    for r in reqs:
        got, iters = results[r.rid]
        assert np.array_equal(host(got), _oracle(r)), (r.rid, r.kind, r.n, tile)
        assert iters == _alone(dl, r)[1], (r.rid, r.kind, r.n, tile)


def test_batch_tune(dl):
    """The grouped-step autotuner returns a tile size and three positive
    times per size, installs its table, and a stream afterwards is still
    exact; bad tables are rejected."""
    import torch

    from paper_1608_00139_amd.serve import run_stream

    b = dl.Batch(pool_bytes=1 << 30, max_active=16, lookahead=1)
    announce("serve tune")
    table = b.tune([100, 700, 1500])
    assert [e["n"] for e in table] == [100, 700, 1500]
    for e in table:
        assert e["tile"] in (64, 128, 256) and all(x > 0 for x in e["ms"])
    reqs = dlgen.serving_stream(10, seed=33, rate=0.0, n_lo=64, n_hi=1500)

    def edges_of(r):
        return torch.from_numpy(dlgen.request_edges(r).astype(np.int32)).cuda()

    stats, results = run_stream(reqs, edges_of, pool_bytes=0, keep_results=True, batch=b)
    for r in reqs:
        assert np.array_equal(host(results[r.rid][0]), _oracle(r)), (r.rid, r.kind, r.n)
    with pytest.raises(dl.DLError):
        b.set_tiles([{"n": 500, "tile": 64}, {"n": 400, "tile": 128}])  # sizes must ascend
    with pytest.raises(dl.DLError):
        b.set_tiles([{"n": 500, "tile": 96}])
    b.set_tiles([])  # back to the built-in rule
    b.close()


def test_lookahead_switch(dl):
    """Look-ahead can be turned off only when no round is in flight; values
    other than 0 and 1 are rejected."""
    b = dl.Batch(pool_bytes=1 << 26, max_active=4)
    lib = dl.load()
    assert lib.dl_batch_set_lookahead(b._h, 2) == 1
    assert lib.dl_batch_set_lookahead(b._h, 1) == 0
    a = dev(np.eye(64, k=1, dtype=np.uint8))
    slot = b.dl_batch_submit(b.TC, a, 0)
    assert slot is not None
    announce("serve lookahead switch")
    b.dl_batch_step()  # round 1 in flight
    assert lib.dl_batch_set_lookahead(b._h, 0) == 1
    iters = None
    for _ in range(20):
        active, _ = b.dl_batch_step()
        for tag, sl, it in b.dl_batch_poll():
            iters = it
            b.dl_batch_fetch(sl)
        if active == 0 and iters is not None:
            break
    b.dl_batch_step()  # drains the round issued before the last completion
    assert lib.dl_batch_set_lookahead(b._h, 0) == 0
    assert iters == dl.dl_tc(a, method=dl.DL_TC_SQUARE)[1]
    b.close()


@pytest.mark.parametrize("lookahead", [0, 1])
def test_large_requests_all_tile_sizes(dl, lookahead):
    """A mix spanning the three tile sizes (n up to 1600: 64, 128 and 256 x 256
    grouped tiles in one round), dense and edge-list admission, against the oracle."""
    import torch

    from paper_1608_00139_amd.serve import run_stream

    reqs = dlgen.serving_stream(14, seed=21, rate=0.0, n_lo=100, n_hi=1600)
    assert any(r.n > 1024 for r in reqs) and any(r.n <= 256 for r in reqs)

    def edges_of(r):
        return torch.from_numpy(dlgen.request_edges(r).astype(np.int32)).cuda()

    announce("serve large", [r.n for r in reqs], lookahead)
    for mk in (edges_of, _make_input):
        stats, results = run_stream(reqs, mk, pool_bytes=1 << 31, max_active=8, keep_results=True,
                                    lookahead=lookahead)
        for r in reqs:
            got, iters = results[r.rid]
            assert np.array_equal(host(got), _oracle(r)), (r.rid, r.kind, r.n)
            assert iters == _alone(dl, r)[1], (r.rid, r.kind, r.n)


@pytest.mark.parametrize("lookahead", [0, 1])
def test_prefetch_across_requests(dl, lookahead):
    """Ten requests of 1100 .. 2048 constants on 256 x 256 tiles: a round
    holds up to 461 tiles for 256 workgroups, so workgroups take a second
    tile, often of another request with another size, whose first slice they
    fetch during the first tile's epilogue.  Every model and iteration count
    is checked."""
    import torch

    from paper_1608_00139_amd.serve import run_stream

    reqs = dlgen.serving_stream(10, seed=41, rate=0.0, n_lo=1100, n_hi=2048)
    assert sum(((r.n + 255) // 256) ** 2 for r in reqs) > 256
    assert len({(r.n + 255) // 256 for r in reqs}) > 2

    def edges_of(r):
        return torch.from_numpy(dlgen.request_edges(r).astype(np.int32)).cuda()

    announce("serve prefetch", [r.n for r in reqs], lookahead)
    stats, results = run_stream(reqs, edges_of, pool_bytes=1 << 31, max_active=16, keep_results=True,
                                lookahead=lookahead, tiles=[{"n": 16384, "tile": 256}])
    for r in reqs:
        got, iters = results[r.rid]
        assert np.array_equal(host(got), _oracle(r)), (r.rid, r.kind, r.n)
        assert iters == _alone(dl, r)[1], (r.rid, r.kind, r.n)


def test_config_serving_stream_10000(dl):
    """The serving configuration as the benchmark runs it: 10,000 requests
    (70% closure on ER p = 3/n, 30% same generation on forests, n
    log-uniform in [64, 2048]) admitted as device edge lists into an 8 GiB
    pool with 512 slots, one round of look-ahead and the autotuned tile
    table.  Every request finishes; a sample of 104 (every 97th) is
    compared with the oracle's model and iteration count."""
    import torch

    from paper_1608_00139_amd.serve import run_stream

    reqs = dlgen.serving_stream(10000, seed=0, rate=0.0)
    flat, offs = [], [0]
    for r in reqs:
        e = dlgen.request_edges(r).astype(np.int32)
        flat.append(e)
        offs.append(offs[-1] + len(e))
    edges = torch.from_numpy(np.concatenate(flat)).cuda()

    def mk(r):
        return edges[offs[r.rid]:offs[r.rid + 1]]

    tb = dl.Batch(1 << 20, 4)
    tiles = tb.tune()
    tb.close()
    sample = set(range(0, len(reqs), 97))
    announce("serve config 10000", len(sample))
    stats, results = run_stream(reqs, mk, pool_bytes=8 << 30, max_active=512, keep_results=sample,
                                lookahead=1, tiles=tiles)
    assert len(stats.completions) == len(reqs)
    assert sorted(c.tag for c in stats.completions) == list(range(len(reqs)))
    by_tag = {c.tag: c for c in stats.completions}
    for rid in sorted(sample):
        r = reqs[rid]
        a = dlgen.to_dense(r.n, dlgen.request_edges(r))
        got, iters = results[rid]
        if r.kind == "tc":
            ref = oracle.tc_seminaive(a)[0]
            _, hist = oracle.bfs(a, want_matrix=False)
            it_ref = oracle.square_schedule_from_hist(hist)[0]
        else:
            ref, _, it_ref, _ = oracle.sg_seminaive(a)
        assert np.array_equal(host(got), ref), (rid, r.kind, r.n)
        assert iters == it_ref, (rid, r.kind, r.n)
        assert by_tag[rid].ones == int(ref.sum()), (rid, r.kind, r.n)


@pytest.mark.parametrize("lookahead", [0, 1])
def test_bulk_admission_and_release(dl, lookahead):
    """dl_batch_submit_edges_n admits the prefix of requests that fits (here
    the slots run out), an invalid request stops it with an error after the
    valid ones before it, and dl_batch_release_n reports the same model sizes
    as dl_batch_fetch; every model equals the oracle's."""
    import torch

    reqs = dlgen.serving_stream(9, seed=21, rate=0.0, n_lo=64, n_hi=400)
    edges = [torch.from_numpy(dlgen.request_edges(r).astype(np.int32)).cuda() for r in reqs]
    kinds = [dl.Batch.TC if r.kind == "tc" else dl.Batch.SG for r in reqs]
    b = dl.Batch(pool_bytes=1 << 28, max_active=6, lookahead=lookahead)
    announce("bulk admission", lookahead)
    slots = b.dl_batch_submit_edges_n(kinds, [r.n for r in reqs], edges, [r.rid for r in reqs])
    assert len(slots) == 6 and len(set(slots)) == 6  # six slots
    with pytest.raises(dl.DLError):
        bad = torch.zeros((1, 2), dtype=torch.int32, device="cuda")
        b.dl_batch_submit_edges_n([dl.Batch.TC], [0], [bad], [99])  # n = 0 is invalid
    fetched, released = {}, {}
    while len(fetched) + len(released) < 6:
        b.dl_batch_step()
        done = b.dl_batch_poll()
        keep = [(tag, sl, it) for tag, sl, it in done if tag % 2 == 0]
        drop = [(tag, sl, it) for tag, sl, it in done if tag % 2 == 1]
        for tag, sl, it in keep:
            r = reqs[tag]
            out = torch.empty((r.n, r.n), dtype=torch.uint8, device="cuda")
            b.dl_batch_fetch(sl, out)
            fetched[tag] = (host(out), it)
        for (tag, sl, it), ones in zip(drop, b.dl_batch_release_n([sl for _, sl, _ in drop])):
            released[tag] = (ones, it)
    for tag, (model, it) in fetched.items():
        assert np.array_equal(model, _oracle(reqs[tag])), tag
    for tag, (ones, it) in released.items():
        assert ones == int(_oracle(reqs[tag]).sum()), tag
    # the remaining three fit now
    slots = b.dl_batch_submit_edges_n(kinds[6:], [r.n for r in reqs[6:]], edges[6:], [r.rid for r in reqs[6:]])
    assert len(slots) == 3
    left = set(range(6, 9))
    while left:
        b.dl_batch_step()
        for tag, sl, it in b.dl_batch_poll():
            r = reqs[tag]
            out = torch.empty((r.n, r.n), dtype=torch.uint8, device="cuda")
            b.dl_batch_fetch(sl, out)
            assert np.array_equal(host(out), _oracle(r)), tag
            left.discard(tag)
    b.close()
