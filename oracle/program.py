"""Layered evaluation of linear binary Datalog programs -- CPU oracle.

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and the bench's CPU leg,
never by the product library, and sharing no code with it.

What it computes (each step with the passage it follows):

* A program is a set of clauses over binary predicates.  Every clause body is
  a chain of atoms from the head's first argument to its second, each atom
  possibly written with its arguments swapped and possibly negated
  (``not p(X,Y)``).  ``eq`` is equality over the n constants (the diag facts
  of Sec. 7.2).  A conjunction along a chain is the relational composition
  of its atoms (Sec. 5: a conjunction of lower-layer atoms becomes a product
  of matrices); a swapped atom is the converse relation (Sec. 6.2); a negated
  atom is the complement over the n x n constant pairs (Sec. 8).
* Strata are the strongly connected components of the predicate dependency
  graph (Sec. 5).  Here a component is found from its plain definition --
  p and q are in one component iff each reaches the other in the dependency
  graph -- by a Boolean closure of the (small) predicate graph, not by
  Tarjan's algorithm, and components are taken in an order where every
  component comes after those it depends on.
* Each component is evaluated by naive bottom-up iteration with its lower
  components fixed: R_h^(0) = 0 and R_h^(k+1) = T_h(R^(k)) for every head h
  of the component at once (the simultaneous series of Sec. 5), until an
  application changes nothing.  ``iters`` counts applications including
  that last one.  The least model of a linear component is reached this way
  (Sec. 5, the lemma on the series of a layer); negated atoms refer to lower
  components only (stratified negation, Sec. 8), which ``evaluate`` checks.

Relations are dense uint8 n x n arrays, row = first argument (Sec. 2).
Compositions use an integer matrix product followed by ``> 0``.
"""
from __future__ import annotations

import re
from dataclasses import dataclass, field

import numpy as np

_TOKEN = re.compile(r"\s*(?:(%[^\n]*)|(:-)|(\\\+)|([A-Za-z_][A-Za-z0-9_]*)|([(),.]))")


@dataclass
class Atom:
    pred: str
    args: tuple
    neg: bool = False


@dataclass
class Clause:
    head: Atom
    body: list = field(default_factory=list)


class ProgramError(ValueError):
    pass


def parse(text: str) -> list:
    """Clauses of ``text``: ``head(X,Y) :- atom, not atom, ... .``  Lines from
    ``%`` on are comments; ``\\+`` is accepted for ``not``."""
    toks = []
    pos = 0
    while pos < len(text):
        m = _TOKEN.match(text, pos)
        if not m or m.end() == pos:
            if text[pos:].strip() == "":
                break
            raise ProgramError(f"unexpected character at offset {pos}")
        pos = m.end()
        if m.group(1):
            continue
        tok = m.group(2) or m.group(3) or m.group(4) or m.group(5)
        toks.append(tok)
    clauses = []
    i = 0

    def atom():
        nonlocal i
        neg = False
        if toks[i] in ("not", "\\+"):
            neg = True
            i += 1
        name = toks[i]
        if not re.fullmatch(r"[a-z][A-Za-z0-9_]*", name):
            raise ProgramError(f"bad predicate name {name!r}")
        if toks[i + 1] != "(" or toks[i + 3] != "," or toks[i + 5] != ")":
            raise ProgramError(f"predicate {name} must be binary")
        a, b = toks[i + 2], toks[i + 4]
        for v in (a, b):
            if not re.fullmatch(r"[A-Z][A-Za-z0-9_]*", v):
                raise ProgramError(f"argument {v!r} is not a variable")
        i += 6
        return Atom(name, (a, b), neg)

    try:
        while i < len(toks):
            head = atom()
            if head.neg:
                raise ProgramError("negated head")
            body = []
            if toks[i] == ":-":
                i += 1
                body.append(atom())
                while toks[i] == ",":
                    i += 1
                    body.append(atom())
            if toks[i] != ".":
                raise ProgramError("missing '.'")
            i += 1
            if not body:
                raise ProgramError("facts are given as relations, not clauses")
            clauses.append(Clause(head, body))
    except IndexError:
        raise ProgramError("unexpected end of program") from None
    return clauses


def _relation(name, neg, rels, n):
    if name == "eq":
        m = np.eye(n, dtype=bool)
    else:
        m = rels[name].astype(bool)
    return ~m if neg else m


def _chain(clause: Clause):
    """The body as a path from the head's first variable to its second:
    a list of (atom, forward) where forward means the atom is read in its
    written argument order."""
    x, z = clause.head.args
    if x == z:
        raise ProgramError("head arguments must be two different variables")
    left = list(clause.body)
    cur, path = x, []
    while left:
        nxt = [a for a in left if cur in a.args]
        if len(nxt) != 1:
            raise ProgramError("body is not a chain from the first head argument to the second")
        a = nxt[0]
        left.remove(a)
        if a.args[0] == a.args[1]:
            raise ProgramError("atom with a repeated variable")
        fwd = a.args[0] == cur
        path.append((a, fwd))
        cur = a.args[1] if fwd else a.args[0]
        if cur == x or (cur == z and left):
            raise ProgramError("body is not a chain from the first head argument to the second")
    if cur != z:
        raise ProgramError("body does not end at the second head argument")
    return path


def _compose(path, rels, n):
    out = None
    for a, fwd in path:
        m = _relation(a.pred, a.neg, rels, n)
        if not fwd:
            m = m.T
        if out is None:
            out = m
        else:
            out = (out.astype(np.float64) @ m.astype(np.float64)) > 0
    return out


def components(clauses):
    """SCCs of the IDB predicates in dependency order (lower first)."""
    idb = sorted({c.head.pred for c in clauses})
    ix = {p: k for k, p in enumerate(idb)}
    m = len(idb)
    dep = np.zeros((m, m), dtype=bool)
    for c in clauses:
        for a in c.body:
            if a.pred in ix:
                dep[ix[c.head.pred], ix[a.pred]] = True
    reach = dep.copy()
    for k in range(m):  # Warshall on the predicate graph
        reach |= reach[:, k:k + 1] & reach[k:k + 1, :]
    same = (reach & reach.T) | np.eye(m, dtype=bool)
    comps, seen = [], set()
    for p in range(m):
        if p in seen:
            continue
        members = [q for q in range(m) if same[p, q]]
        seen.update(members)
        comps.append(members)
    # order: a component depends only on components placed before it
    ordered, placed = [], set()
    while len(ordered) < len(comps):
        for comp in comps:
            if comp[0] in placed:
                continue
            deps = {q for p in comp for q in range(m) if reach[p, q] and not same[p, q]}
            if deps <= placed:
                ordered.append(comp)
                placed.update(comp)
    return [[idb[k] for k in comp] for comp in ordered], reach, ix


def evaluate(text: str, edb: dict, n: int):
    """Least (perfect) model of the program.  Returns (model, layers) where
    model maps every IDB predicate to its uint8 relation and layers lists, in
    evaluation order, (sorted head names, iters)."""
    clauses = parse(text)
    comps, reach, ix = components(clauses)
    heads = {c.head.pred for c in clauses}
    for c in clauses:
        for a in c.body:
            if a.pred != "eq" and a.pred not in heads and a.pred not in edb:
                raise ProgramError(f"relation {a.pred} is neither defined nor given")
    if "eq" in heads:
        raise ProgramError("eq is built in")
    for name in edb:
        if name in heads:
            raise ProgramError(f"{name} is defined by clauses and also given")
    rels = {k: (np.asarray(v) != 0) for k, v in edb.items()}
    layers = []
    for comp in comps:
        cs = set(comp)
        mine = [c for c in clauses if c.head.pred in cs]
        for c in mine:
            rec = [a for a in c.body if a.pred in cs]
            if len(rec) > 1:
                raise ProgramError(f"clause for {c.head.pred} is not linear")
            for a in c.body:
                if a.neg and a.pred in ix and reach[ix[a.pred], ix[c.head.pred]]:
                    raise ProgramError(f"negation of {a.pred} is not stratified")
        paths = [(c.head.pred, _chain(c)) for c in mine]
        cur = {h: np.zeros((n, n), dtype=bool) for h in comp}
        iters = 0
        while True:
            env = dict(rels)
            env.update(cur)
            nxt = {h: np.zeros((n, n), dtype=bool) for h in comp}
            for h, path in paths:
                nxt[h] |= _compose(path, env, n)
            iters += 1
            if all(np.array_equal(nxt[h], cur[h]) for h in comp):
                break
            cur = nxt
        rels.update(cur)
        layers.append((sorted(comp), iters))
    model = {h: rels[h].astype(np.uint8) for h in heads}
    return model, layers
