"""The serving loop's host logic (paper_1608_00139_amd.serve.run_stream) on the
CPU, against a stand-in batch that finishes each request after a known number
of rounds: every request completes exactly once, none is admitted before it
arrives, admission waits while slots or pool memory are taken, and a request
larger than an empty pool is an error.  (The device side of the same loop is
covered by the GPU serving tests.)"""
from __future__ import annotations

import pytest
import torch

import dlgen
from paper_1608_00139_amd.serve import run_stream


class StandInBatch:
    """Slots and pool bytes as the library accounts them (4 n^2 bytes per
    request); request `tag` finishes after 1 + n % 5 rounds."""

    TC, SG = 0, 1

    def __init__(self, slots: int, pool_bytes: int):
        self.slots = [None] * slots
        self.pool = pool_bytes
        self.used = 0
        self.finished: list[int] = []
        self.rounds = 0
        self.admitted: list[int] = []

    def _admit(self, tag: int, n: int):
        need = 4 * n * n
        if self.used + need > self.pool:
            return None
        for i, s in enumerate(self.slots):
            if s is None:
                self.slots[i] = {"tag": tag, "left": 1 + n % 5, "bytes": need}
                self.used += need
                self.admitted.append(tag)
                return i
        return None

    def dl_batch_submit_edges(self, kind: int, n: int, edges: torch.Tensor, tag: int):
        assert edges.dtype == torch.int32 and edges.dim() == 2 and edges.shape[1] == 2
        return self._admit(tag, n)

    def dl_batch_submit(self, kind: int, rel: torch.Tensor, tag: int):
        return self._admit(tag, rel.shape[0])

    def dl_batch_step(self):
        self.rounds += 1
        for i, s in enumerate(self.slots):
            if s is not None and s["left"] > 0:
                s["left"] -= 1
                if s["left"] == 0:
                    self.finished.append(i)
        return sum(1 for s in self.slots if s is not None and s["left"] > 0), 0

    def dl_batch_poll(self):
        out = [(self.slots[i]["tag"], i, 7) for i in self.finished]
        self.finished = []
        return out

    def dl_batch_fetch(self, slot: int, out=None) -> int:
        s = self.slots[slot]
        assert s is not None and s["left"] == 0, "fetch of an unfinished or free slot"
        self.used -= s["bytes"]
        self.slots[slot] = None
        return 11


class StandInBulkBatch(StandInBatch):
    """The same, with the bulk admission and release calls (admission stops
    at the first request that does not fit)."""

    def __init__(self, slots: int, pool_bytes: int):
        super().__init__(slots, pool_bytes)
        self.bulk_calls = 0

    def dl_batch_submit_edges_n(self, kinds, ns, edges, tags):
        self.bulk_calls += 1
        assert len(kinds) == len(ns) == len(edges) == len(tags)
        out = []
        for n, e, tag in zip(ns, edges, tags):
            assert e.dtype == torch.int32 and e.dim() == 2 and e.shape[1] == 2
            slot = self._admit(tag, n)
            if slot is None:
                break
            out.append(slot)
        return out

    def dl_batch_release_n(self, slots):
        return [self.dl_batch_fetch(s) for s in slots]


BATCHES = [StandInBatch, StandInBulkBatch]


def _edges(req):
    return torch.from_numpy(dlgen.request_edges(req)).to(torch.int32)


@pytest.mark.parametrize("cls", BATCHES)
def test_burst_every_request_once(cls):
    reqs = dlgen.serving_stream(60, seed=3, rate=0.0, n_lo=64, n_hi=300)
    b = cls(slots=8, pool_bytes=1 << 30)
    stats, results = run_stream(reqs, _edges, pool_bytes=0, batch=b)
    tags = sorted(c.tag for c in stats.completions)
    assert tags == list(range(60)) and sorted(b.admitted) == tags
    assert results == {}
    assert stats.eagain > 0 and stats.max_active == 8  # more requests than slots
    assert b.used == 0 and all(s is None for s in b.slots)
    for c in stats.completions:
        assert c.arrival <= c.admitted <= c.finished and c.iters == 7 and c.ones == 11


@pytest.mark.parametrize("cls", BATCHES)
def test_pool_memory_limits_admission(cls):
    reqs = dlgen.serving_stream(30, seed=4, rate=0.0, n_lo=200, n_hi=300)
    pool = 3 * 4 * 300 * 300  # room for about three requests at a time
    b = cls(slots=16, pool_bytes=pool)
    stats, _ = run_stream(reqs, _edges, pool_bytes=0, batch=b)
    assert len(stats.completions) == 30
    assert stats.max_active <= pool // (4 * min(r.n for r in reqs) ** 2) and stats.eagain > 0


@pytest.mark.parametrize("cls", BATCHES)
def test_arrivals_are_respected(cls):
    reqs = dlgen.serving_stream(40, seed=5, rate=4000.0, n_lo=64, n_hi=128)
    assert reqs[-1].arrival > 0.0
    b = cls(slots=4, pool_bytes=1 << 30)
    stats, _ = run_stream(reqs, _edges, pool_bytes=0, batch=b)
    assert len(stats.completions) == 40
    for c in stats.completions:
        assert c.admitted >= c.arrival  # never admitted before it arrives


@pytest.mark.parametrize("cls", BATCHES)
def test_request_larger_than_the_pool(cls):
    reqs = dlgen.serving_stream(3, seed=6, rate=0.0, n_lo=500, n_hi=600)
    b = cls(slots=4, pool_bytes=4 * 100 * 100)
    with pytest.raises(RuntimeError, match="does not fit an empty pool"):
        run_stream(reqs, _edges, pool_bytes=0, batch=b)


def test_burst_admitted_in_chunks():
    """A burst larger than the admission chunk is admitted a chunk per round,
    with one bulk call per chunk, while the earlier requests run."""
    reqs = dlgen.serving_stream(50, seed=7, rate=0.0, n_lo=64, n_hi=100)
    b = StandInBulkBatch(slots=64, pool_bytes=1 << 30)
    stats, _ = run_stream(reqs, _edges, pool_bytes=0, batch=b, admit_chunk=16)
    assert sorted(c.tag for c in stats.completions) == list(range(50))
    assert b.bulk_calls == 4  # 16 + 16 + 16 + 2
    first = sorted(c.admitted for c in stats.completions)
    assert first[15] < first[16]  # the second chunk came after a round
