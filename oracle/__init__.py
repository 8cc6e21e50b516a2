"""CPU oracle for the linear-algebraic Datalog evaluation hot path.

TEST INFRASTRUCTURE ONLY.  The oracle is imported by ``tests/``, by the smoke
check and by the bench's CPU-baseline leg; the product library never imports,
links or calls it, and it shares no code with the GPU path.

What it computes, each piece with the passage it follows:

* ``tc_seminaive`` -- least model of the transitive-closure program DB1
  (Sec. 3), by semi-naive iteration of T_DB (Sec. 2) in C on bitset rows.
  Because DB1 is linear, the facts after round k equal the matrix iterate
  R^(k) of the series R^(0)=0, R^(k+1)=min1(R1 + R1 R^(k)) (Sec. 3), so
  the per-round counts double as per-step counts of that series.
* ``tc_seminaive_edges`` -- the same rounds from an edge list, with the
  rounds alone timed (the CPU baseline's timed region).
* ``tc_square_literal`` -- the series R^(k+1)=min1(R1 + R^(k) R^(k)) of the
  non-linear closure program in Sec. 8, step by step with Boolean rows.
* ``bfs`` -- one breadth-first search per source: reachability and the
  histogram of shortest path lengths (length >= 1).  Brute force in the
  spirit of the paper's Warshall cross-check (Sec. 7.1).
* ``warshall`` -- Warshall's algorithm (Sec. 7.1).
* ``sg_seminaive`` -- least model of the same-generation program (Sec. 7.2,
  equation R2 = min1(I + R1 R2 R1^T)), semi-naive in C.
* ``eps_solve`` -- the purely linear form of Sec. 4, Proposition 1:
  X = (I - eps R1)^-1 eps R1, as one fp64 LAPACK solve.
* ``eps_solve_exact`` -- the same X in exact rational arithmetic (plain
  Gauss-Jordan elimination on Fractions), for tiny n.
* ``naive_tdb`` -- textbook naive bottom-up evaluation of a Datalog program
  over sets of ground atoms (Sec. 2), for tiny inputs; it pins the matrix
  forms to the logic.
* ``sg_eps_kron`` -- the same-generation epsilon equation
  X = eps (I + R1 X R1^T) solved through the vec/Kronecker form of Sec. 6.3
  (O(n^6): tiny n only).
* ``linear_solve`` -- the tail-recursive equation X = eps (C + B X) of
  Sec. 6.1 as one fp64 LAPACK solve.
* ``two_sided_kron`` -- the two-sided equation X = eps (Q + B X C) of
  Sec. 6.3 through its vec/Kronecker form (tiny n only).
* ``oracle.program`` -- layered evaluation of linear programs (its own
  module header says what it follows).

Conventions: relations are dense n x n arrays, row = first argument (Sec. 2),
nonzero = true; results are uint8 0/1.  ``ones[k]`` is the number of true
entries of iterate k (k = 0..iters); ``iters`` counts applications of the
update from the empty relation, including the first one that changes nothing.
"""
from __future__ import annotations

import ctypes
import os
from fractions import Fraction
from itertools import product as _iproduct

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None
_default_threads = 1


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b

            _b.build()
        lib = ctypes.CDLL(_LIB_PATH)
        i64 = ctypes.c_int64
        pu8 = ctypes.c_void_p
        pi64 = ctypes.c_void_p
        for name in ("or_tc_seminaive", "or_tc_square_literal", "or_sg_seminaive"):
            f = getattr(lib, name)
            f.argtypes = [i64, pu8, pu8, pi64, i64, pi64]
            f.restype = ctypes.c_int
        lib.or_warshall.argtypes = [i64, pu8, pu8]
        lib.or_warshall.restype = ctypes.c_int
        lib.or_bfs.argtypes = [i64, pu8, pi64, i64, pu8, pi64]
        lib.or_bfs.restype = ctypes.c_int
        lib.or_num_threads.argtypes = []
        lib.or_num_threads.restype = ctypes.c_int
        lib.or_tc_seminaive_edges.argtypes = [i64, i64, ctypes.c_void_p, ctypes.c_int, pu8, pi64, pi64,
                                              ctypes.c_void_p, ctypes.c_void_p]
        lib.or_tc_seminaive_edges.restype = ctypes.c_int
        global _default_threads
        _default_threads = int(lib.or_num_threads())
        _lib = lib
    return _lib


def num_threads() -> int:
    return int(_load().or_num_threads())


def default_threads() -> int:
    """OpenMP's thread count when the library was loaded (OMP_NUM_THREADS,
    else every core the process may use): the all-core setting."""
    _load()
    return _default_threads


def _as_u8(a) -> np.ndarray:
    a = np.asarray(a)
    if a.ndim != 2 or a.shape[0] != a.shape[1]:
        raise ValueError("relation must be a square matrix")
    return np.ascontiguousarray(a != 0, dtype=np.uint8)


def _ptr(x: np.ndarray):
    return ctypes.c_void_p(x.ctypes.data)


def _check(rc: int, name: str) -> None:
    if rc == 2:
        raise MemoryError(f"{name}: allocation failed")
    if rc == 3:
        raise ValueError(f"{name}: bad arguments")


def _iterate(fn_name: str, a, maxsteps: int | None):
    a = _as_u8(a)
    n = a.shape[0]
    cap = (n * n + 2) if maxsteps is None else int(maxsteps)
    ones_len = min(cap, n * n + 2) + 2
    ones = np.zeros(ones_len, dtype=np.int64)
    out = np.zeros((n, n), dtype=np.uint8)
    iters = np.zeros(1, dtype=np.int64)
    rc = getattr(_load(), fn_name)(n, _ptr(a), _ptr(out), _ptr(ones), cap, _ptr(iters))
    _check(rc, fn_name)
    k = int(iters[0])
    return out, ones[: k + 1].copy(), k, rc == 0


def tc_seminaive(a, maxsteps: int | None = None):
    """Closure of ``a`` by semi-naive T_DB; returns (R, ones, iters, converged).

    With ``maxsteps=k`` (k smaller than the convergence step) R is the k-th
    iterate R^(k) of the plain series and ``converged`` is False.
    """
    return _iterate("or_tc_seminaive", a, maxsteps)


def tc_seminaive_edges(n: int, edges, threads: int = 0, want_model: bool = True):
    """Closure of the relation given as an edge list ([m, 2] pairs (i, j)),
    by the same semi-naive rounds as ``tc_seminaive``, with the rounds timed
    alone (set-up and the dense copy of the model are outside the clock).

    ``threads`` > 0 sets the OpenMP thread count (it stays set for later
    oracle calls); 0 restores the count the library was loaded with.
    Returns (R or None, iters, model ones, seconds, threads used).
    """
    threads = int(threads) if threads > 0 else default_threads()
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
    out = np.zeros((n, n), dtype=np.uint8) if want_model else None
    ones = np.zeros(1, dtype=np.int64)
    iters = np.zeros(1, dtype=np.int64)
    secs = np.zeros(1, dtype=np.float64)
    used = np.zeros(1, dtype=np.int32)
    rc = _load().or_tc_seminaive_edges(n, e.shape[0], _ptr(e) if e.size else None, threads,
                                       None if out is None else _ptr(out), _ptr(ones), _ptr(iters),
                                       _ptr(secs), _ptr(used))
    _check(rc, "or_tc_seminaive_edges")
    return out, int(iters[0]), int(ones[0]), float(secs[0]), int(used[0])


def tc_square_literal(a, maxsteps: int | None = None):
    """Series R^(k+1) = min1(A + R^(k) R^(k)) taken literally (Boolean rows)."""
    return _iterate("or_tc_square_literal", a, maxsteps)


def sg_seminaive(p, maxsteps: int | None = None):
    """Same-generation model of parent relation ``p``; (S, ones, iters, converged)."""
    return _iterate("or_sg_seminaive", p, maxsteps)


def warshall(a) -> np.ndarray:
    a = _as_u8(a)
    n = a.shape[0]
    out = np.zeros((n, n), dtype=np.uint8)
    _check(_load().or_warshall(n, _ptr(a), _ptr(out)), "or_warshall")
    return out


def bfs(a, rows=None, want_matrix: bool = True):
    """Per-source BFS.  Returns (R_rows or None, hist).

    ``hist[L]`` counts pairs (s, t) over the chosen sources whose shortest
    path of length >= 1 has length L.  ``R_rows[i]`` is the reachability row
    of source ``rows[i]`` (all sources when ``rows`` is None).
    """
    a = _as_u8(a)
    n = a.shape[0]
    if rows is None:
        rows_arr = None
        ns = n
    else:
        rows_arr = np.ascontiguousarray(rows, dtype=np.int64)
        ns = rows_arr.size
    hist = np.zeros(n + 2, dtype=np.int64)
    out = np.zeros((ns, n), dtype=np.uint8) if want_matrix else None
    rc = _load().or_bfs(n, _ptr(a), None if rows_arr is None else _ptr(rows_arr), ns,
                        None if out is None else _ptr(out), _ptr(hist))
    _check(rc, "or_bfs")
    return out, hist


def max_path_length(hist: np.ndarray) -> int:
    """D = largest shortest-path length over reachable pairs (0 if none)."""
    nz = np.nonzero(hist)[0]
    return int(nz[-1]) if nz.size else 0


def plain_schedule_from_hist(hist: np.ndarray):
    """(iters, ones) of the plain series from a full path-length histogram.

    R^(k) holds exactly the pairs joined by a path of length in [1, k], so
    ones[k] = sum_{L<=k} hist[L] and the series first repeats at step D+1.
    """
    d = max_path_length(hist)
    iters = d + 1
    ones = np.array([int(hist[1:k + 1].sum()) for k in range(iters + 1)], dtype=np.int64)
    return iters, ones


def square_schedule_from_hist(hist: np.ndarray):
    """(iters, ones) of the squaring series from a full path-length histogram.

    R^(k) (k >= 1) holds exactly the pairs joined by a path of length in
    [1, 2^(k-1)]: a shortest path of length L <= 2^k, L >= 2, splits in two
    paths of length <= 2^(k-1) each.  So the series first repeats at step
    1 if D = 0, else 2 + ceil(log2 D).
    """
    d = max_path_length(hist)
    if d == 0:
        iters = 1
    else:
        iters = 2 + int(np.ceil(np.log2(d))) if d > 1 else 2
    ones = [0]
    for k in range(1, iters + 1):
        lim = min(2 ** (k - 1), len(hist) - 1)
        ones.append(int(hist[1:lim + 1].sum()))
    return iters, np.array(ones, dtype=np.int64)


def eps_bound(a) -> float:
    """Largest eps allowed by Lemma 1: 1 / (1 + ||R1||_inf), ||.||_inf = max row sum."""
    a = _as_u8(a)
    return 1.0 / (1.0 + float(a.sum(axis=1).max(initial=0)))


def eps_solve(a, eps: float) -> np.ndarray:
    """X = (I - eps A)^-1 eps A in fp64 (Proposition 1), one LAPACK solve."""
    a = _as_u8(a).astype(np.float64)
    n = a.shape[0]
    if n == 0:
        return np.zeros((0, 0))
    return np.linalg.solve(np.eye(n) - eps * a, eps * a)


def eps_solve_exact(a, eps: Fraction) -> list[list[Fraction]]:
    """Exact rational X with (I - eps A) X = eps A, by Gauss-Jordan elimination.

    Written independently of LAPACK: row operations on the augmented matrix
    [I - eps A | eps A] over Fractions, pivoting on the first nonzero entry.
    """
    a = _as_u8(a)
    n = a.shape[0]
    eps = Fraction(eps)
    m = [[(Fraction(1) if i == j else Fraction(0)) - eps * int(a[i, j]) for j in range(n)]
         + [eps * int(a[i, j]) for j in range(n)] for i in range(n)]
    for c in range(n):
        piv = next(r for r in range(c, n) if m[r][c] != 0)
        m[c], m[piv] = m[piv], m[c]
        pv = m[c][c]
        m[c] = [x / pv for x in m[c]]
        for r in range(n):
            if r != c and m[r][c] != 0:
                f = m[r][c]
                m[r] = [x - f * y for x, y in zip(m[r], m[c])]
    return [row[n:] for row in m]


def naive_tdb(facts: set, rules: list) -> set:
    """Least Herbrand model by naive bottom-up evaluation (Sec. 2).

    ``facts`` is a set of ground atoms (pred, c1, c2); ``rules`` is a list of
    (head, body) where head and body atoms are (pred, var_or_const, ...) and
    variables are strings starting with an upper-case letter.  I^(0) is
    empty and I^(n+1) = T_DB(I^(n)); the loop returns the first repeated
    interpretation.  Exponential in the body length: tiny inputs only.
    """
    consts = sorted({c for f in facts for c in f[1:]})

    def is_var(t):
        return isinstance(t, str) and t[:1].isupper()

    def ground(rule_vars, env, atom):
        return (atom[0],) + tuple(env[t] if is_var(t) else t for t in atom[1:])

    interp: set = set()
    while True:
        new = set(facts)
        for head, body in rules:
            vs = sorted({t for atom in (head, *body) for t in atom[1:] if is_var(t)})
            for vals in _iproduct(consts, repeat=len(vs)):
                env = dict(zip(vs, vals))
                if all(ground(vs, env, b) in interp for b in body):
                    new.add(ground(vs, env, head))
        if new == interp:
            return interp
        interp = new


def sg_forest_closed_form(parents: np.ndarray) -> np.ndarray:
    """Same-generation model of a forest given as (child, parent) rows.

    (x, w) holds iff x and w have the same depth and the same root.
    """
    n = parents.size
    depth = np.zeros(n, dtype=np.int64)
    root = np.arange(n)
    for i in range(n):  # parents[i] < i, so one forward pass suffices
        p = parents[i]
        if p >= 0:
            depth[i] = depth[p] + 1
            root[i] = root[p]
    return ((depth[:, None] == depth[None, :]) & (root[:, None] == root[None, :])).astype(np.uint8)


def sg_eps_kron(p, eps: float) -> np.ndarray:
    """Solve X = eps (I + P X P^T) through vec(X) = eps (vec(I) + (P kron P) vec(X)).

    Uses vec(A X B) = (B^T kron A) vec(X) (Sec. 2, Sec. 6.3): with B = P^T,
    B^T kron A = P kron P.  O(n^6) -- tiny n only.
    """
    pm = _as_u8(p).astype(np.float64)
    n = pm.shape[0]
    k = np.kron(pm, pm)
    vec_i = np.eye(n).reshape(-1, order="F")
    x = np.linalg.solve(np.eye(n * n) - eps * k, eps * vec_i)
    return x.reshape((n, n), order="F")


def linear_solve(b, c, eps: float) -> np.ndarray:
    """Tail-recursive equation X = eps (C + B X) (Sec. 6.1) as one fp64 LAPACK
    solve of (I - eps B) X = eps C."""
    bm = _as_u8(b).astype(np.float64)
    cm = _as_u8(c).astype(np.float64)
    n = bm.shape[0]
    return np.linalg.solve(np.eye(n) - eps * bm, eps * cm)


def two_sided_kron(q, b, c, eps: float) -> np.ndarray:
    """Two-sided equation X = eps (Q + B X C) (Sec. 6.3) through
    vec(X) = eps (vec(Q) + (C^T kron B) vec(X)), using vec(B X C) =
    (C^T kron B) vec(X).  O(n^6): tiny n only."""
    qm = _as_u8(q).astype(np.float64)
    bm = _as_u8(b).astype(np.float64)
    cm = _as_u8(c).astype(np.float64)
    n = qm.shape[0]
    k = np.kron(cm.T, bm)
    x = np.linalg.solve(np.eye(n * n) - eps * k, eps * qm.reshape(-1, order="F"))
    return x.reshape((n, n), order="F")
