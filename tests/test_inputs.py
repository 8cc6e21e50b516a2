"""The seeded generators: determinism, shape and the stated distributions."""
from __future__ import annotations

import numpy as np

import dlgen


def test_er_deterministic_and_well_formed():
    n = 500
    e1 = dlgen.er_edges(n, 4.0 / n, 7)
    e2 = dlgen.er_edges(n, 4.0 / n, 7)
    assert np.array_equal(e1, e2)
    assert dlgen.edges_sha256(n, e1) == dlgen.edges_sha256(n, e2)
    assert not np.array_equal(e1, dlgen.er_edges(n, 4.0 / n, 8))
    assert e1.dtype == np.int32 and e1.shape[1] == 2
    assert np.all(e1[:, 0] != e1[:, 1])
    assert np.all((e1 >= 0) & (e1 < n))
    key = e1[:, 0].astype(np.int64) * n + e1[:, 1]
    assert np.all(np.diff(key) > 0)  # sorted, no duplicates
    # mean edge count n(n-1)p = 1996; 6 sigma window
    assert abs(len(e1) - 4.0 * (n - 1)) < 6 * np.sqrt(4.0 * (n - 1))


def test_er_extremes_and_self_loops():
    assert len(dlgen.er_edges(10, 0.0, 0)) == 0
    assert len(dlgen.er_edges(10, 1.0, 0)) == 90
    assert len(dlgen.er_edges(10, 1.0, 0, self_loops=True)) == 100
    e = dlgen.er_edges(200, 0.2, 3, self_loops=True)
    assert np.any(e[:, 0] == e[:, 1])


def test_forest_shape():
    n = 4096
    par = dlgen.forest_parents(n, 0)
    assert par[0] == -1
    i = np.arange(1, n)
    nonroot = par[1:] >= 0
    assert np.all(par[1:][nonroot] < i[nonroot])
    frac_root = 1 - nonroot.mean()
    assert 0.08 < frac_root < 0.12
    e = dlgen.forest_edges(n, 0)
    a = dlgen.to_dense(n, e)
    assert a.sum(axis=1).max() == 1  # one parent per child


def test_chung_lu_shape():
    n = 2000
    e = dlgen.chung_lu_edges(n, 0)
    assert np.array_equal(e, dlgen.chung_lu_edges(n, 0))
    assert np.all(e[:, 0] != e[:, 1])
    key = e[:, 0].astype(np.int64) * n + e[:, 1]
    assert np.all(np.diff(key) > 0)
    mean = len(e) / n
    assert 5.0 < mean < 8.5  # the min(1, .) cap lowers the realized mean below 8
    deg = np.bincount(e[:, 0], minlength=n)
    assert deg[:10].mean() > 10 * deg[-1000:].mean()  # heavy head


def test_serving_stream():
    rs = dlgen.serving_stream(2000, 0, rate=100.0)
    assert len(rs) == 2000
    ns = np.array([r.n for r in rs])
    assert ns.min() >= 64 and ns.max() <= 2048
    frac_tc = np.mean([r.kind == "tc" for r in rs])
    assert 0.66 < frac_tc < 0.74
    arr = np.array([r.arrival for r in rs])
    assert np.all(np.diff(arr) >= 0)
    assert 15 < arr[-1] < 25
