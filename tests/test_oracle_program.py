"""Pins of the layered program oracle (oracle/program.py) against things other
than itself: textbook naive T_DB over ground atoms (rules written out here as
tuples, not parsed by the oracle), the transitive-closure and same-generation
oracles, a walk-parity brute force, and stratum-by-stratum ground evaluation
for negation."""
from __future__ import annotations

import itertools

import numpy as np
import pytest

import dlgen
import oracle
from oracle import program as prog


def _facts(rels: dict, n: int) -> set:
    f = {("eq", c, c) for c in range(n)}  # also fixes the domain to all n constants
    for name, m in rels.items():
        for i, j in zip(*np.nonzero(m)):
            f.add((name, int(i), int(j)))
    return f


def _matrix(model: set, name: str, n: int) -> np.ndarray:
    out = np.zeros((n, n), dtype=np.uint8)
    for atom in model:
        if atom[0] == name:
            out[atom[1], atom[2]] = 1
    return out


def _rand(n, p, seed, loops=True):
    return dlgen.to_dense(n, dlgen.er_edges(n, p, seed, self_loops=loops))


# Each case: program text, the same rules as tuples for naive T_DB, EDB names.
CASES = {
    "tc_right": (
        "tc(X,Z) :- e(X,Z).\ntc(X,Z) :- e(X,Y), tc(Y,Z).",
        [(("tc", "X", "Z"), [("e", "X", "Z")]), (("tc", "X", "Z"), [("e", "X", "Y"), ("tc", "Y", "Z")])],
        ["e"],
    ),
    "tc_left": (
        "tc(X,Z) :- e(X,Z).\ntc(X,Z) :- tc(X,Y), e(Y,Z).",
        [(("tc", "X", "Z"), [("e", "X", "Z")]), (("tc", "X", "Z"), [("tc", "X", "Y"), ("e", "Y", "Z")])],
        ["e"],
    ),
    "sg": (
        "sg(X,Y) :- eq(X,Y).\nsg(X,Y) :- p(X,U), sg(U,V), p(Y,V).",
        [(("sg", "X", "Y"), [("eq", "X", "Y")]),
         (("sg", "X", "Y"), [("p", "X", "U"), ("sg", "U", "V"), ("p", "Y", "V")])],
        ["p"],
    ),
    "transposed": (  # Sec. 6.2 example: r2(x,z) <- r1(x,y), r2(z,y)
        "r2(X,Z) :- r1(X,Z).\nr2(X,Z) :- r1(X,Y), r2(Z,Y).",
        [(("r2", "X", "Z"), [("r1", "X", "Z")]), (("r2", "X", "Z"), [("r1", "X", "Y"), ("r2", "Z", "Y")])],
        ["r1"],
    ),
    "two_sided": (  # Sec. 6.3 example: r2(x,z) <- r1(x,y), r2(y,w), r3(w,z)
        "r2(X,Z) :- r1(X,Z).\nr2(X,Z) :- r1(X,Y), r2(Y,W), r3(W,Z).",
        [(("r2", "X", "Z"), [("r1", "X", "Z")]),
         (("r2", "X", "Z"), [("r1", "X", "Y"), ("r2", "Y", "W"), ("r3", "W", "Z")])],
        ["r1", "r3"],
    ),
    "even_odd": (
        "odd(X,Z) :- e(X,Z).\nodd(X,Z) :- e(X,Y), even(Y,Z).\neven(X,Z) :- e(X,Y), odd(Y,Z).",
        [(("odd", "X", "Z"), [("e", "X", "Z")]), (("odd", "X", "Z"), [("e", "X", "Y"), ("even", "Y", "Z")]),
         (("even", "X", "Z"), [("e", "X", "Y"), ("odd", "Y", "Z")])],
        ["e"],
    ),
    "layers": (  # three layers: closure, a product with it, a recursion over that
        "tc(X,Z) :- e(X,Z).\ntc(X,Z) :- e(X,Y), tc(Y,Z).\n"
        "q(X,Z) :- f(Y,X), tc(Y,Z).\n"
        "w(X,Z) :- q(X,Z).\nw(X,Z) :- w(X,Y), f(Y,Z).",
        [(("tc", "X", "Z"), [("e", "X", "Z")]), (("tc", "X", "Z"), [("e", "X", "Y"), ("tc", "Y", "Z")]),
         (("q", "X", "Z"), [("f", "Y", "X"), ("tc", "Y", "Z")]),
         (("w", "X", "Z"), [("q", "X", "Z")]), (("w", "X", "Z"), [("w", "X", "Y"), ("f", "Y", "Z")])],
        ["e", "f"],
    ),
    "mixed_general": (  # two recursive clauses for one head: neither tail form nor one Stein term
        "r(X,Z) :- a(X,Z).\nr(X,Z) :- b(X,Y), r(Y,Z).\nr(X,Z) :- r(X,Y), c(Y,Z).\nr(X,Z) :- b(X,Y), r(W,Y), c(W,Z).",
        [(("r", "X", "Z"), [("a", "X", "Z")]), (("r", "X", "Z"), [("b", "X", "Y"), ("r", "Y", "Z")]),
         (("r", "X", "Z"), [("r", "X", "Y"), ("c", "Y", "Z")]),
         (("r", "X", "Z"), [("b", "X", "Y"), ("r", "W", "Y"), ("c", "W", "Z")])],
        ["a", "b", "c"],
    ),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_program_vs_naive_tdb(name):
    text, rules, edbs = CASES[name]
    for seed in range(6):
        n = 3 + seed % 3
        rels = {e: _rand(n, 0.3, 10 * seed + k) for k, e in enumerate(edbs)}
        model, _ = prog.evaluate(text, rels, n)
        ground = oracle.naive_tdb(_facts(rels, n), rules)
        for head in model:
            assert np.array_equal(model[head], _matrix(ground, head, n)), (name, seed, head)


def test_tc_programs_match_closure_oracle_and_iters():
    for seed in range(3):
        n = 150
        a = _rand(n, 1.5 / n, seed, loops=False)
        ref, _, iters, _ = oracle.tc_seminaive(a)
        m, layers = prog.evaluate(CASES["tc_right"][0], {"e": a}, n)
        assert np.array_equal(m["tc"], ref) and layers == [(["tc"], iters)]
        m, layers = prog.evaluate(CASES["tc_left"][0], {"e": a}, n)
        assert np.array_equal(m["tc"], ref) and layers == [(["tc"], iters)]


def test_sg_program_matches_sg_oracle_and_iters():
    for seed in range(3):
        n = 120
        p = dlgen.to_dense(n, dlgen.forest_edges(n, seed))
        ref, _, iters, _ = oracle.sg_seminaive(p)
        m, layers = prog.evaluate(CASES["sg"][0], {"p": p}, n)
        assert np.array_equal(m["sg"], ref) and layers == [(["sg"], iters)]


def test_even_odd_walk_parity_bruteforce():
    """odd/even = pairs joined by a walk of odd/even length >= 1 (BFS on the
    node x parity graph)."""
    for seed in range(4):
        n = 40
        e = _rand(n, 2.0 / n, seed, loops=False)
        m, layers = prog.evaluate(CASES["even_odd"][0], {"e": e}, n)
        odd = np.zeros((n, n), np.uint8)
        even = np.zeros((n, n), np.uint8)
        adj = [np.nonzero(e[i])[0] for i in range(n)]
        for s in range(n):
            seen = set()
            frontier = [(int(j), 1) for j in adj[s]]
            while frontier:
                nxt = []
                for v, par in frontier:
                    if (v, par) in seen:
                        continue
                    seen.add((v, par))
                    nxt.extend((int(w), 1 - par) for w in adj[v])
                frontier = nxt
            for v, par in seen:
                (odd if par else even)[s, v] = 1
        assert np.array_equal(m["odd"], odd) and np.array_equal(m["even"], even)
        assert len(layers) == 1 and layers[0][0] == ["even", "odd"]


NEG_TEXT = """
tc(X,Y) :- e(X,Y).
tc(X,Y) :- e(X,Z), tc(Z,Y).
nr(X,Y) :- not tc(X,Y).
r(X,Z) :- e(X,Y), not tc(Y,Z).
s(X,Z) :- f(X,Z).
s(X,Z) :- s(X,Y), not e(Y,Z).
"""


def test_stratified_negation_vs_ground_strata():
    """Negation: lower stratum first, then its complement as ground facts
    (the perfect model of a stratified program, Sec. 8)."""
    for seed in range(6):
        n = 3 + seed % 3
        e = _rand(n, 0.35, seed)
        f = _rand(n, 0.3, 100 + seed)
        model, layers = prog.evaluate(NEG_TEXT, {"e": e, "f": f}, n)
        base = _facts({"e": e, "f": f}, n)
        tc_rules = [(("tc", "X", "Y"), [("e", "X", "Y")]), (("tc", "X", "Y"), [("e", "X", "Z"), ("tc", "Z", "Y")])]
        low = oracle.naive_tdb(base, tc_rules)
        tc = _matrix(low, "tc", n)
        comp = {("ntc", i, j) for i, j in itertools.product(range(n), repeat=2) if not tc[i, j]}
        comp |= {("ne", i, j) for i, j in itertools.product(range(n), repeat=2) if not e[i, j]}
        upper = [(("nr", "X", "Y"), [("ntc", "X", "Y")]), (("r", "X", "Z"), [("e", "X", "Y"), ("ntc", "Y", "Z")]),
                 (("s", "X", "Z"), [("f", "X", "Z")]), (("s", "X", "Z"), [("s", "X", "Y"), ("ne", "Y", "Z")])]
        high = oracle.naive_tdb(base | low | comp, upper)
        for h in ("nr", "r", "s"):
            assert np.array_equal(model[h], _matrix(high, h, n)), (seed, h)
        assert np.array_equal(model["tc"], tc)
        assert [l[0] for l in layers].index(["tc"]) < [l[0] for l in layers].index(["r"])


@pytest.mark.parametrize("text,msg", [
    ("t(X,Z) :- e(X,Z).\nt(X,Z) :- t(X,Y), t(Y,Z).", "not linear"),
    ("p(X,Y) :- e(X,Y), not e(X,Y).", "not a chain"),
    ("p(X,Y) :- e(X,Y).\nq(X,Y) :- e(X,Z), not p(Z,Y).\np(X,Y) :- q(X,Y).", "not stratified"),
    ("p(X,Y) :- e(X,Z), e(Z,Z), e(Z,Y).", "not a chain"),
    ("p(X,X) :- e(X,X).", "two different"),
    ("eq(X,Y) :- e(X,Y).", "built in"),
    ("p(X,Y) :- g(X,Y).", "neither defined"),
    ("p(X,Y) :- e(X,a).", "not a variable"),
    ("p(X,Y) :- e(X,Y)", "end of program"),
])
def test_program_errors(text, msg):
    with pytest.raises(prog.ProgramError, match=msg):
        prog.evaluate(text, {"e": np.eye(3, dtype=np.uint8)}, 3)


def test_planted_mistake_ignoring_argument_order_fails(monkeypatch):
    """An oracle that reads every atom in written order fails the naive T_DB pin."""
    real = prog._chain

    def sloppy(clause):
        return [(a, True) for a, _ in real(clause)]

    monkeypatch.setattr(prog, "_chain", sloppy)
    text, rules, edbs = CASES["transposed"]
    bad = 0
    for seed in range(6):
        n = 4
        rels = {"r1": _rand(n, 0.3, seed)}
        model, _ = prog.evaluate(text, rels, n)
        ground = oracle.naive_tdb(_facts(rels, n), rules)
        bad += not np.array_equal(model["r2"], _matrix(ground, "r2", n))
    assert bad > 0


# ---------------------------------------------------------------- the epsilon forms of Sec. 6


def test_linear_solve_threshold_residual_and_rationals():
    """X = eps (C + B X): [X > 0] = C + TC(B) C (the Boolean least solution,
    from the closure oracle), residual at rounding level, and exact rational
    elimination on tiny inputs."""
    from fractions import Fraction

    for seed in range(5):
        n = 6 + 7 * seed
        b = _rand(n, 2.0 / n, seed)
        c = _rand(n, 1.5 / n, 50 + seed)
        eps = 1.0 / (1 + int(b.sum(axis=1).max()))
        x = oracle.linear_solve(b, c, eps)
        tcb = oracle.tc_seminaive(b)[0].astype(np.int64)
        want = ((c.astype(np.int64) + tcb @ c.astype(np.int64)) > 0).astype(np.uint8)
        assert np.array_equal((x > 0).astype(np.uint8), want)
        bf, cf = b.astype(np.float64), c.astype(np.float64)
        assert np.abs(x - eps * (cf + bf @ x)).max() < 1e-14
        if n <= 13:
            e = Fraction(eps).limit_denominator(1000)
            m = [[Fraction(int(i == j)) - e * int(b[i, j]) for j in range(n)] + [e * int(c[i, j]) for j in range(n)]
                 for i in range(n)]
            for k in range(n):  # plain Gauss-Jordan on rationals
                piv = m[k][k]
                m[k] = [v / piv for v in m[k]]
                for i in range(n):
                    if i != k and m[i][k] != 0:
                        f = m[i][k]
                        m[i] = [vi - f * vk for vi, vk in zip(m[i], m[k])]
            exact = np.array([[float(m[i][n + j]) for j in range(n)] for i in range(n)])
            assert np.allclose(x, exact, rtol=1e-13, atol=1e-16)


TWO_SIDED_TEXT = "r(X,Z) :- q(X,Z).\nr(X,Z) :- b(X,Y), r(Y,W), c(W,Z)."


def test_two_sided_kron_threshold_series_and_residual():
    """X = eps (Q + B X C): [X > 0] equals the layered oracle's model of the
    matching two-sided program, X equals the partial sums of
    eps sum_m eps^m B^m Q C^m, and the residual is at rounding level."""
    for seed in range(5):
        n = 4 + seed
        q = _rand(n, 0.2, seed)
        b = _rand(n, 0.3, 20 + seed)
        c = _rand(n, 0.3, 40 + seed)
        nb = int(b.sum(axis=1).max())
        nc = int(c.sum(axis=0).max())
        eps = 1.0 / (1 + nb * nc)
        x = oracle.two_sided_kron(q, b, c, eps)
        model, _ = prog.evaluate(TWO_SIDED_TEXT, {"q": q, "b": b, "c": c}, n)
        assert np.array_equal((x > 0).astype(np.uint8), model["r"])
        qf, bf, cf = (m.astype(np.float64) for m in (q, b, c))
        series, term = np.zeros((n, n)), eps * qf
        for _ in range(4000):
            series += term
            term = eps * (bf @ term @ cf)
        assert np.allclose(x, series, rtol=1e-10, atol=1e-15)
        assert np.abs(x - eps * (qf + bf @ x @ cf)).max() < 1e-14
