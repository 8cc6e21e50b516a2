"""Pins for the CPU oracle: each checks it against something other than itself.

Sources of truth used here: the worked example printed at the end of Sec. 4,
Warshall's algorithm and per-source BFS (the paper's own cross-check in
Sec. 7.1), textbook naive T_DB evaluation over ground atoms (Sec. 2), closed
forms for special graphs, exact rational arithmetic, and the lemmas of Sec. 4
as invariants.
"""
from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np
import pytest

import dlgen
import oracle
from tests.golden.load import load_sections

pytestmark = pytest.mark.filterwarnings("ignore")


def _tc_rules():
    # DB1 of Sec. 3: r2(X,Z) <- r1(X,Z).  r2(X,Z) <- r1(X,Y), r2(Y,Z).
    return [(("r2", "X", "Z"), [("r1", "X", "Z")]),
            (("r2", "X", "Z"), [("r1", "X", "Y"), ("r2", "Y", "Z")])]


def _sg_rules():
    # Same-generation program of Sec. 7.2.
    return [(("r2", "X", "W"), [("diag", "X", "W")]),
            (("r2", "X", "W"), [("r1", "X", "Y"), ("r2", "Y", "Z"), ("r1", "W", "Z")])]


def _model_matrix(model, pred, n):
    m = np.zeros((n, n), dtype=np.uint8)
    for atom in model:
        if atom[0] == pred:
            m[atom[1], atom[2]] = 1
    return m


def _facts(a, pred="r1"):
    return {(pred, int(i), int(j)) for i, j in zip(*np.nonzero(a))}


def _literal_plain_series(a, k):
    """R^(k) of R^(j+1) = min1(A + A R^(j)) with a library integer matmul."""
    a = a.astype(np.int64)
    r = np.zeros_like(a)
    for _ in range(k):
        r = ((a + a @ r) > 0).astype(np.int64)
    return r.astype(np.uint8)


# ---------------------------------------------------------------- worked example


def test_worked_example_values_and_model():
    g = load_sections("worked_example.txt")
    a = g["R1"].astype(np.uint8)
    eps = float(g["eps"][0, 0])
    assert eps == oracle.eps_bound(a) == 0.5
    exact = oracle.eps_solve_exact(a, Fraction(1, 2))
    # the printed digits are truncations of sevenths
    sev = {Fraction(1, 7), Fraction(2, 7), Fraction(4, 7), Fraction(0)}
    assert all(x in sev for row in exact for x in row)
    xf = np.array([[float(x) for x in row] for row in exact])
    assert np.all(np.abs(xf - g["X_printed"]) < 1e-4)
    assert np.all(np.floor(xf * 1e4) / 1e4 == g["X_printed"])
    x64 = oracle.eps_solve(a, eps)
    assert np.allclose(x64, xf, rtol=1e-14, atol=1e-15)
    r2 = g["R2_printed"].astype(np.uint8)
    assert np.array_equal((x64 > 0).astype(np.uint8), r2)
    r, ones, iters, conv = oracle.tc_seminaive(a)
    assert conv and np.array_equal(r, r2)
    # path lengths: D = 3, so the plain series repeats at step 4
    assert iters == 4 and list(ones) == [0, 4, 8, 12, 12]
    rs, ones_s, iters_s, _ = oracle.tc_square_literal(a)
    assert np.array_equal(rs, r2) and iters_s == 4


# ---------------------------------------------------------------- exhaustive brute force


def test_tc_all_3node_digraphs_with_self_loops():
    """All 2^9 relations on 3 constants: semi-naive == Warshall == BFS == naive T_DB."""
    n = 3
    for bits in range(1 << 9):
        a = np.array([(bits >> b) & 1 for b in range(9)], dtype=np.uint8).reshape(3, 3)
        r, ones, iters, conv = oracle.tc_seminaive(a)
        assert conv
        w = oracle.warshall(a)
        b, hist = oracle.bfs(a)
        model = oracle.naive_tdb(_facts(a), _tc_rules())
        t = _model_matrix(model, "r2", n)
        assert np.array_equal(r, w) and np.array_equal(r, b) and np.array_equal(r, t), bits
        it_p, ones_p = oracle.plain_schedule_from_hist(hist)
        assert iters == it_p and np.array_equal(ones, ones_p), bits
        rs, ones_s, iters_s, conv_s = oracle.tc_square_literal(a)
        it_s, ones_ss = oracle.square_schedule_from_hist(hist)
        assert conv_s and np.array_equal(rs, r) and iters_s == it_s and np.array_equal(ones_s, ones_ss), bits


def test_tc_all_4node_digraphs_no_self_loops():
    n = 4
    offd = [(i, j) for i in range(n) for j in range(n) if i != j]
    for bits in range(1 << len(offd)):
        a = np.zeros((n, n), dtype=np.uint8)
        for b, (i, j) in enumerate(offd):
            a[i, j] = (bits >> b) & 1
        r, ones, iters, _ = oracle.tc_seminaive(a)
        b_, hist = oracle.bfs(a)
        assert np.array_equal(r, oracle.warshall(a)) and np.array_equal(r, b_)
        it_p, ones_p = oracle.plain_schedule_from_hist(hist)
        assert iters == it_p and np.array_equal(ones, ones_p)
        rs, _, iters_s, _ = oracle.tc_square_literal(a)
        assert np.array_equal(rs, r) and iters_s == oracle.square_schedule_from_hist(hist)[0]


@pytest.mark.parametrize("n,p,seed", [(5, 0.3, 0), (7, 0.2, 1), (16, 0.1, 2), (33, 0.05, 3),
                                      (64, 2 / 64, 4), (64, 0.2, 5), (64, 1.0, 6), (1, 0.5, 7)])
def test_tc_random_vs_bruteforce(n, p, seed):
    for loops in (False, True):
        a = dlgen.to_dense(n, dlgen.er_edges(n, p, seed, self_loops=loops))
        r, ones, iters, conv = oracle.tc_seminaive(a)
        assert conv
        assert np.array_equal(r, oracle.warshall(a))
        b, hist = oracle.bfs(a)
        assert np.array_equal(r, b)
        it_p, ones_p = oracle.plain_schedule_from_hist(hist)
        assert iters == it_p and np.array_equal(ones, ones_p)
        # per-step parity of the semi-naive rounds with the literal matrix series
        for k in range(0, iters + 1):
            rk, ok, _, _ = oracle.tc_seminaive(a, maxsteps=k)
            assert np.array_equal(rk, _literal_plain_series(a, k)), (n, p, k)
            assert int(rk.sum()) == ones[k]
        rs, ones_s, iters_s, _ = oracle.tc_square_literal(a)
        it_s, ones_ss = oracle.square_schedule_from_hist(hist)
        assert np.array_equal(rs, r) and iters_s == it_s and np.array_equal(ones_s, ones_ss)


@pytest.mark.parametrize("n,p,seed", [(0, 0.0, 0), (1, 0.5, 1), (40, 0.06, 2), (257, 1.5 / 257, 3),
                                      (600, 4 / 600, 4)])
def test_tc_edge_list_entry_vs_bfs(n, p, seed):
    """The edge-list entry (the CPU baseline's timed rounds) against BFS
    reachability and the path-length histogram, with repeated pairs, self
    loops and out-of-range pairs in the list, at one thread and at all."""
    e = dlgen.er_edges(n, p, seed, self_loops=True) if n else np.zeros((0, 2), np.int64)
    junk = np.array([[-1, 0], [0, n], [n, n + 3]], np.int64)
    lst = np.concatenate([e, e[: len(e) // 2], junk]) if n else junk
    a = dlgen.to_dense(n, e) if n else np.zeros((0, 0), np.uint8)
    if n:
        ref, hist = oracle.bfs(a)
        it_ref = oracle.plain_schedule_from_hist(hist)[0]
    else:
        ref, it_ref = np.zeros((0, 0), np.uint8), 1
    for threads in (1, 0):
        r, iters, ones, secs, used = oracle.tc_seminaive_edges(n, lst, threads=threads)
        assert np.array_equal(r, ref) and iters == it_ref and ones == int(ref.sum())
        assert secs >= 0.0 and used >= 1
    assert oracle.tc_seminaive_edges(n, lst, threads=1)[4] == 1
    assert oracle.tc_seminaive_edges(0, np.zeros((0, 2), np.int32))[4] == oracle.default_threads()


def test_tc_naive_tdb_random_small():
    for seed in range(20):
        n = 2 + seed % 4
        a = dlgen.to_dense(n, dlgen.er_edges(n, 0.35, seed, self_loops=True))
        t = _model_matrix(oracle.naive_tdb(_facts(a), _tc_rules()), "r2", n)
        assert np.array_equal(oracle.tc_seminaive(a)[0], t)


def test_bfs_sampled_rows_match_full():
    n = 200
    a = dlgen.to_dense(n, dlgen.er_edges(n, 1.5 / n, 11))
    full, hist = oracle.bfs(a)
    rows = np.array([0, 17, 199, 5, 5])
    part, _ = oracle.bfs(a, rows=rows)
    assert np.array_equal(part, full[rows])


# ---------------------------------------------------------------- closed forms


def test_tc_closed_forms():
    # empty relation: nothing derivable; the first update already repeats
    for n in (1, 5, 64):
        r, ones, iters, _ = oracle.tc_seminaive(np.zeros((n, n), np.uint8))
        assert r.sum() == 0 and iters == 1 and list(ones) == [0, 0]
        assert oracle.tc_square_literal(np.zeros((n, n), np.uint8))[2] == 1
    # complete digraph without loops: all pairs, (i,i) needs a 2-cycle -> D = 2
    for n in (2, 3, 9):
        a = 1 - np.eye(n, dtype=np.uint8)
        r, ones, iters, _ = oracle.tc_seminaive(a)
        assert r.all() and iters == 3
        assert oracle.tc_square_literal(a)[2] == 3
    # directed cycle: everything, D = n
    for n in (2, 5, 13, 64):
        a = np.roll(np.eye(n, dtype=np.uint8), 1, axis=1)
        r, ones, iters, _ = oracle.tc_seminaive(a)
        assert r.all() and iters == n + 1
        assert oracle.tc_square_literal(a)[2] == 2 + int(np.ceil(np.log2(n)))
    # directed path: strictly upper triangle, D = n - 1
    for n in (2, 6, 40):
        a = np.eye(n, k=1, dtype=np.uint8)
        r, ones, iters, _ = oracle.tc_seminaive(a)
        assert np.array_equal(r, np.triu(np.ones((n, n), np.uint8), 1)) and iters == n
        assert list(ones) == [0] + [sum(n - d for d in range(1, k + 1)) for k in range(1, n)] + [n * (n - 1) // 2]


def test_tc_forest_is_proper_ancestor_relation():
    n = 300
    par = dlgen.forest_parents(n, 3)
    a = dlgen.to_dense(n, dlgen.forest_edges(n, 3))
    anc = np.zeros((n, n), np.uint8)
    for i in range(n):
        p = par[i]
        while p >= 0:
            anc[i, p] = 1
            p = par[p]
    assert np.array_equal(oracle.tc_seminaive(a)[0], anc)


# ---------------------------------------------------------------- same generation


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (10, 2), (100, 3), (513, 4)])
def test_sg_forest_closed_form(n, seed):
    par = dlgen.forest_parents(n, seed)
    p = dlgen.to_dense(n, dlgen.forest_edges(n, seed))
    s, ones, iters, conv = oracle.sg_seminaive(p)
    assert conv
    assert np.array_equal(s, oracle.sg_forest_closed_form(par))
    # fixpoint equation S = min1(I + P S P^T) and symmetry
    s64 = s.astype(np.int64)
    p64 = p.astype(np.int64)
    assert np.array_equal(s, ((np.eye(n, dtype=np.int64) + p64 @ s64 @ p64.T) > 0).astype(np.uint8))
    assert np.array_equal(s, s.T)
    # reversed orientation (first argument = parent): only the diagonal, repeats at step 2
    pr = dlgen.to_dense(n, dlgen.forest_edges(n, seed, child_to_parent=False))
    sr, _, it_r, _ = oracle.sg_seminaive(pr)
    assert np.array_equal(sr, np.eye(n, dtype=np.uint8)) and it_r == 2


def test_sg_naive_tdb_random_small():
    for seed in range(16):
        n = 2 + seed % 3
        p = dlgen.to_dense(n, dlgen.er_edges(n, 0.4, seed, self_loops=True))
        facts = _facts(p) | {("diag", i, i) for i in range(n)}
        # make every constant visible to the evaluator's domain
        facts |= {("dom", i, i) for i in range(n)}
        t = _model_matrix(oracle.naive_tdb(facts, _sg_rules()), "r2", n)
        assert np.array_equal(oracle.sg_seminaive(p)[0], t), seed


def test_sg_per_step_matches_literal_series():
    n = 40
    p = dlgen.to_dense(n, dlgen.er_edges(n, 0.06, 9, self_loops=True))
    s, ones, iters, _ = oracle.sg_seminaive(p)
    p64 = p.astype(np.int64)
    cur = np.zeros((n, n), np.int64)
    for k in range(1, iters + 1):
        cur = ((np.eye(n, dtype=np.int64) + p64 @ cur @ p64.T) > 0).astype(np.int64)
        sk, ok, _, _ = oracle.sg_seminaive(p, maxsteps=k)
        assert np.array_equal(sk, cur.astype(np.uint8)) and int(cur.sum()) == ones[k]


# ---------------------------------------------------------------- epsilon form


def _dist_matrix(a):
    """dist(i,j) = first step k at which R^(k)_ij = 1 (0 if never)."""
    r, ones, iters, _ = oracle.tc_seminaive(a)
    d = np.zeros(a.shape, np.int64)
    for k in range(iters, 0, -1):
        rk = oracle.tc_seminaive(a, maxsteps=k)[0]
        d[rk == 1] = k
    return d


@pytest.mark.parametrize("seed", range(6))
def test_eps_exact_rationals_vs_fp64_and_theorem1(seed):
    n = 3 + seed
    a = dlgen.to_dense(n, dlgen.er_edges(n, 0.3, seed, self_loops=True))
    d_inf = int(a.sum(axis=1).max())
    for eps in (Fraction(1, 1 + d_inf), Fraction(1, 2 * (1 + d_inf))):
        ex = oracle.eps_solve_exact(a, eps)
        xf = np.array([[float(v) for v in row] for row in ex])
        x64 = oracle.eps_solve(a, float(eps))
        assert np.allclose(x64, xf, rtol=1e-12, atol=1e-14)
        # Theorem 1: thresholding the exact least solution gives the closure
        thr = np.array([[1 if v > 0 else 0 for v in row] for row in ex], np.uint8)
        assert np.array_equal(thr, oracle.tc_seminaive(a)[0])
        # Lemma 1: 0 <= X <= 1; exact fixpoint of X = eps (A + A X)
        assert all(0 <= v <= 1 for row in ex for v in row)
        for i in range(n):
            for j in range(n):
                rhs = eps * (int(a[i, j]) + sum(int(a[i, m]) * ex[m][j] for m in range(n)))
                assert rhs == ex[i][j]
        # footnote to Lemma 2: a pair first derived at step k has X >= eps^k
        dist = _dist_matrix(a)
        for i in range(n):
            for j in range(n):
                if dist[i, j]:
                    assert ex[i][j] >= eps ** int(dist[i, j])


def test_eps_cycle_values_closed_form():
    """Directed cycle C_n: X_ij = sum over walks = eps^L / (1 - eps^n), L = (j-i) mod n or n."""
    n = 6
    a = np.roll(np.eye(n, dtype=np.uint8), 1, axis=1)
    eps = 0.5
    x = oracle.eps_solve(a, eps)
    for i in range(n):
        for j in range(n):
            L = (j - i) % n or n
            assert abs(x[i, j] - eps ** L / (1 - eps ** n)) < 1e-15


def test_sg_eps_kron_threshold_and_residual():
    for seed in range(4):
        n = 5 + seed
        p = dlgen.to_dense(n, dlgen.forest_edges(n, seed))
        d = int(p.sum(axis=1).max())
        eps = 1.0 / (1 + d * d)
        x = oracle.sg_eps_kron(p, eps)
        assert np.array_equal((x > 0).astype(np.uint8), oracle.sg_seminaive(p)[0])
        pf = p.astype(np.float64)
        assert np.allclose(x, eps * (np.eye(n) + pf @ x @ pf.T), atol=1e-14)
        assert np.allclose(x, x.T, atol=1e-15)


# ---------------------------------------------------------------- planted mistakes


def test_pins_catch_transposed_operand():
    """A plausible oracle bug (joining on the wrong side) must fail the worked example."""
    g = load_sections("worked_example.txt")
    a = g["R1"].astype(np.uint8)
    wrong = oracle.tc_seminaive(a.T)[0]  # as if the join read r1(y,x)
    assert not np.array_equal(wrong, g["R2_printed"].astype(np.uint8))
    wrong_eps = np.linalg.solve(np.eye(4) - 0.5 * a, 0.5 * a.T)  # transposed right-hand side
    assert not np.allclose(wrong_eps, g["X_printed"], atol=1e-4)


def test_pins_catch_dropped_exit_rule():
    """Dropping the r1 term (R = min1(A R)) must fail the brute-force pin."""
    a = dlgen.to_dense(8, dlgen.er_edges(8, 0.3, 1))
    r = np.zeros((8, 8), np.int64)
    for _ in range(10):
        r = ((a.astype(np.int64) @ r) > 0).astype(np.int64)
    assert not np.array_equal(r.astype(np.uint8), oracle.warshall(a))
