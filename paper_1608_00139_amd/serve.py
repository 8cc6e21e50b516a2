"""Request loop over the batching C ABI: arrivals, admission by pool memory,
one grouped step per round, retirement, latency accounting.

Every product runs in the library's grouped kernel (dl_batch_step); this
module only decides which requests are in the batch.  A request that arrives
while others are on the GPU is admitted as soon as a slot and pool memory are
free, and starts moving with the very next round.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import torch

from . import Batch


@dataclass
class Completion:
    tag: int
    kind: int
    n: int
    iters: int
    ones: int
    arrival: float
    admitted: float
    finished: float

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclass
class StreamStats:
    completions: list = field(default_factory=list)
    rounds: int = 0
    wall: float = 0.0
    max_active: int = 0
    eagain: int = 0

    def summary(self) -> dict:
        lat = sorted(c.latency for c in self.completions)
        n = len(lat)

        def pct(q):
            return lat[min(n - 1, int(round(q * (n - 1))))] if n else None

        return {"requests": n, "wall_s": round(self.wall, 4),
                "req_per_s": round(n / self.wall, 1) if self.wall > 0 else None,
                "p50_ms": round(pct(0.50) * 1e3, 3) if n else None,
                "p99_ms": round(pct(0.99) * 1e3, 3) if n else None,
                "mean_ms": round(sum(lat) / n * 1e3, 3) if n else None,
                "rounds": self.rounds, "max_active": self.max_active, "admission_waits": self.eagain}


def run_stream(requests, make_input, pool_bytes: int, max_active: int = 256, keep_results: bool | set = False,
               batch: Batch | None = None, lookahead: int = 0, tiles: list | None = None,
               admit_chunk: int = 64) -> tuple[StreamStats, dict]:
    """Serve `requests` (objects with rid, kind 'tc'/'sg', n, arrival seconds).

    make_input(req) returns the request's relation as a uint8 device tensor
    (dense n x n) or as a device int32 [m, 2] edge list.  lookahead = 1 lets
    each round's host work overlap the next round on the device.  tiles is a
    tile table (Batch.tune's result) for a batch this call creates.  At most
    admit_chunk requests are admitted between two rounds, so that a burst of
    arrivals is admitted while the device runs the rounds of the requests
    admitted before it (edge-list requests are admitted with one library
    call per group).
    Returns the statistics and, if keep_results, {rid: (model tensor, iters)}
    (keep_results may be a set of rids to keep only those models).
    """
    b = batch or Batch(pool_bytes, max_active, lookahead=lookahead)
    if tiles is not None and batch is None:
        b.set_tiles(tiles)
    bulk = hasattr(b, "dl_batch_submit_edges_n") and hasattr(b, "dl_batch_release_n")
    pending = deque(sorted(requests, key=lambda r: r.arrival))
    waiting: deque = deque()
    inflight = {}  # slot -> (req, admitted time)
    results = {}
    stats = StreamStats()
    t0 = time.perf_counter()
    now = 0.0

    def kind_of(req):
        return Batch.TC if req.kind == "tc" else Batch.SG

    def submit_group(group, rels):
        """Slots of the admitted prefix of `group`."""
        if bulk and all(r.dtype == torch.int32 for r in rels):
            return b.dl_batch_submit_edges_n([kind_of(q) for q in group], [q.n for q in group], rels,
                                             [q.rid for q in group])
        slots = []
        for q, rel in zip(group, rels):
            if rel.dtype == torch.int32:
                slot = b.dl_batch_submit_edges(kind_of(q), q.n, rel, q.rid)
            else:
                slot = b.dl_batch_submit(kind_of(q), rel, q.rid)
            if slot is None:
                break
            slots.append(slot)
        return slots

    while pending or waiting or inflight:
        now = time.perf_counter() - t0
        while pending and pending[0].arrival <= now:
            waiting.append(pending.popleft())
        budget = admit_chunk
        while waiting and budget > 0:
            group = [waiting[i] for i in range(min(budget, len(waiting)))]
            rels = [make_input(q) for q in group]
            slots = submit_group(group, rels)
            if not slots and not inflight:
                # with look-ahead, memory of fetched requests returns to the
                # pool once the round in flight completes
                b.dl_batch_step()
                slots = submit_group(group, rels)
            t_adm = time.perf_counter() - t0
            for q, slot in zip(group, slots):
                waiting.popleft()
                inflight[slot] = (q, t_adm)
            budget -= len(slots)
            if len(slots) < len(group):
                if not slots and not inflight:
                    raise RuntimeError(f"request {group[0].rid} (n={group[0].n}) does not fit an empty pool")
                stats.eagain += 1
                break
        if not inflight:
            if pending:  # idle until the next arrival
                while time.perf_counter() - t0 < pending[0].arrival:
                    pass
            continue
        stats.max_active = max(stats.max_active, len(inflight))
        b.dl_batch_step()
        stats.rounds += 1
        done = b.dl_batch_poll()
        if not done:
            continue
        fin = time.perf_counter() - t0
        keep_of = {}
        for tag, slot, iters in done:
            req = inflight[slot][0]
            keep_of[slot] = (req.rid in keep_results) if isinstance(keep_results, set) else bool(keep_results)
        drop = [slot for _, slot, _ in done if not keep_of[slot]]
        ones_of = dict(zip(drop, b.dl_batch_release_n(drop))) if bulk else {}
        for tag, slot, iters in done:
            req, adm = inflight.pop(slot)
            if keep_of[slot]:
                out = torch.empty((req.n, req.n), dtype=torch.uint8, device="cuda")
                ones = b.dl_batch_fetch(slot, out)
                results[req.rid] = (out, iters)
                t_fin = time.perf_counter() - t0
            else:
                ones = ones_of[slot] if bulk else b.dl_batch_fetch(slot, None)
                t_fin = fin
            stats.completions.append(Completion(tag, 0 if req.kind == "tc" else 1, req.n, iters, ones,
                                                req.arrival, adm, t_fin))
    if torch.cuda.is_available():
        torch.cuda.synchronize()
    stats.wall = time.perf_counter() - t0
    return stats, results
