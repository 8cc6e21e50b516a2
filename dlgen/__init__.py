"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module holds input generation only: graphs as edge lists, the dense 0/1
encoding of an edge list, and the serving request stream.  It contains none of
the evaluation method's arithmetic (no products, thresholds or fixpoints), so
both the CPU oracle and the GPU path can consume its output without sharing
any of the method's code.

Workloads follow the paper's experiments (Sec. 7): Erdos-Renyi matrices where
each entry is one with the edge probability p_e; a random forest for the
same-generation program; and a Chung-Lu power-law digraph that stands in for
the real network datasets of Table "Transitive closure computation for real
datasets", which are not reproduced here.

Every generator uses numpy's PCG64 bit generator with an explicit seed, so the
same call gives the same bytes on every machine.
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "er_edges",
    "forest_parents",
    "forest_edges",
    "chung_lu_edges",
    "worked_example_edges",
    "to_dense",
    "edges_sha256",
    "Request",
    "serving_stream",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def er_edges(n: int, p: float, seed: int, self_loops: bool = False) -> np.ndarray:
    """Directed Erdos-Renyi edge list, int32 [E, 2] sorted row-major.

    Every ordered pair (i, j) is an edge independently with probability p
    (Sec. 7.1).  With ``self_loops=False`` only pairs i != j are drawn.  The
    sampler walks the pair index space in row-major order with geometric
    gaps, so the cost is O(E) rather than O(n^2).
    """
    if n <= 0:
        return np.zeros((0, 2), dtype=np.int32)
    m = n * n if self_loops else n * (n - 1)
    if p <= 0.0 or m == 0:
        return np.zeros((0, 2), dtype=np.int32)
    if p >= 1.0:
        t = np.arange(m, dtype=np.int64)
    else:
        rng = _rng(seed)
        chunks = []
        pos = -1
        expect = int(m * p * 1.1) + 64
        while True:
            gaps = rng.geometric(p, size=expect).astype(np.int64)
            idx = pos + np.cumsum(gaps)
            keep = idx[idx < m]
            chunks.append(keep)
            if keep.size < idx.size:
                break
            pos = int(idx[-1])
        t = np.concatenate(chunks) if chunks else np.zeros(0, dtype=np.int64)
    if self_loops:
        i = t // n
        j = t % n
    else:
        i = t // (n - 1)
        jj = t % (n - 1)
        j = jj + (jj >= i)
    return np.stack([i, j], axis=1).astype(np.int32)


def forest_parents(n: int, seed: int, p_root: float = 0.1) -> np.ndarray:
    """Random forest as a parent array (-1 marks a root).

    Node 0 is a root; node i >= 1 is a root with probability ``p_root``, else
    its parent is uniform in [0, i).  Depth grows like log n.
    """
    rng = _rng(seed)
    par = np.full(n, -1, dtype=np.int64)
    if n > 1:
        hi = np.arange(1, n, dtype=np.int64)
        cand = rng.integers(0, hi)
        is_root = rng.random(n - 1) < p_root
        par[1:] = np.where(is_root, -1, cand)
    return par


def forest_edges(n: int, seed: int, child_to_parent: bool = True) -> np.ndarray:
    """Edge list of the parent relation of ``forest_parents(n, seed)``.

    With ``child_to_parent=True`` the edge is (child, parent): row = child.
    With ``False`` it is (parent, child), the reading where the first argument
    is the parent.
    """
    par = forest_parents(n, seed)
    child = np.nonzero(par >= 0)[0]
    parent = par[child]
    if child_to_parent:
        e = np.stack([child, parent], axis=1)
    else:
        e = np.stack([parent, child], axis=1)
        e = e[np.lexsort((e[:, 1], e[:, 0]))]
    return e.astype(np.int32)


def chung_lu_weights(n: int, gamma: float = 2.1, mean_degree: float = 8.0) -> np.ndarray:
    """Expected-degree weights w_i = c (i+1)^(-1/(gamma-1)), mean = mean_degree."""
    base = np.arange(1, n + 1, dtype=np.float64) ** (-1.0 / (gamma - 1.0))
    return base * (mean_degree * n / base.sum())


def chung_lu_edges(n: int, seed: int, gamma: float = 2.1, mean_degree: float = 8.0) -> np.ndarray:
    """Directed Chung-Lu power-law digraph, int32 [E, 2], no self-loops.

    Pair (i, j), i != j, is an edge with probability min(1, w_i w_j / sum(w))
    using the same weight for the in- and out-role.  Sampled per source row
    with the skip-and-thin method of Miller and Hagberg (2011): weights are in
    decreasing order, so an upper bound on the probability of the rest of the
    row lets the sampler jump with a geometric gap and accept with the ratio
    of the true to the bound probability.  The realized mean degree is below
    ``mean_degree`` where the cap at one bites.
    """
    w = chung_lu_weights(n, gamma, mean_degree)
    s = float(w.sum())
    rng = _rng(seed)
    src = []
    dst = []
    for i in range(n):
        wi = w[i]
        j = 0
        p = min(1.0, wi * w[0] / s)
        while j < n and p > 0.0:
            if p < 1.0:
                r = rng.random()
                j += int(math.floor(math.log(r) / math.log1p(-p))) if r > 0.0 else n
            if j >= n:
                break
            q = min(1.0, wi * w[j] / s)
            if rng.random() < q / p and j != i:
                src.append(i)
                dst.append(j)
            p = q
            j += 1
    e = np.stack([np.asarray(src, dtype=np.int64), np.asarray(dst, dtype=np.int64)], axis=1)
    return e.astype(np.int32)


def worked_example_edges() -> np.ndarray:
    """The four-constant relation of the worked example closing Sec. 4.

    r1(e1,e2), r1(e2,e3), r1(e3,e1), r1(e4,e1), written 0-based.
    """
    return np.array([[0, 1], [1, 2], [2, 0], [3, 0]], dtype=np.int32)


def to_dense(n: int, edges: np.ndarray, dtype=np.uint8) -> np.ndarray:
    """Dense n x n 0/1 matrix with entry (i, j) = 1 for each edge (i, j).

    Row = first argument, the adjacency encoding of Sec. 2.
    """
    a = np.zeros((n, n), dtype=dtype)
    if len(edges):
        a[edges[:, 0], edges[:, 1]] = 1
    return a


def edges_sha256(n: int, edges: np.ndarray) -> str:
    h = hashlib.sha256()
    h.update(np.int64(n).tobytes())
    h.update(np.ascontiguousarray(edges, dtype=np.int32).tobytes())
    return h.hexdigest()


@dataclass
class Request:
    rid: int
    kind: str  # "tc" or "sg"
    n: int
    seed: int
    arrival: float  # seconds since stream start


def serving_stream(count: int, seed: int, rate: float = 0.0, n_lo: int = 64, n_hi: int = 2048,
                   p_tc: float = 0.7) -> list[Request]:
    """Request stream: kind TC with probability p_tc else SG, n log-uniform.

    n = round(exp(U[ln n_lo, ln n_hi])).  Arrivals are a Poisson process of
    ``rate`` requests per second; ``rate <= 0`` means all arrive at time 0
    (a closed burst).  TC requests use ER edge probability 3/n and SG
    requests a random forest; the graph of request k uses seed ``seed*1_000_003 + k``.
    """
    rng = _rng(seed)
    kinds = np.where(rng.random(count) < p_tc, "tc", "sg")
    ns = np.rint(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), size=count))).astype(np.int64)
    if rate > 0:
        arr = np.cumsum(rng.exponential(1.0 / rate, size=count))
    else:
        arr = np.zeros(count)
    return [Request(k, str(kinds[k]), int(ns[k]), seed * 1_000_003 + k, float(arr[k])) for k in range(count)]


def request_edges(req: Request) -> np.ndarray:
    if req.kind == "tc":
        return er_edges(req.n, 3.0 / req.n, req.seed)
    return forest_edges(req.n, req.seed)
