"""Layered program evaluation on the GPU through the C ABI, bit-exact against
the layered oracle; the tail-recursive and two-sided epsilon solvers against
their fp64 oracles."""
from __future__ import annotations

import numpy as np
import pytest

import dlgen
import oracle
from oracle import program as oprog
from tests.gpu_util import announce, dev, gpu, host
from tests.test_oracle_program import CASES, NEG_TEXT, TWO_SIDED_TEXT

pytestmark = gpu

FORMS = {
    "tc_right": ["right_tail"],
    "tc_left": ["left_tail"],
    "sg": ["two_sided"],
    "transposed": ["two_sided"],
    "two_sided": ["two_sided"],
    "even_odd": ["right_tail"],
    "layers": ["right_tail", "nonrecursive", "left_tail"],
    "mixed_general": ["general"],
}


@pytest.fixture(scope="module")
def dl():
    import paper_1608_00139_amd as m

    m.load()
    return m


def _rand(n, p, seed, loops=True):
    return dlgen.to_dense(n, dlgen.er_edges(n, min(p, 1.0), seed, self_loops=loops))


def _run(dl, text, rels, n, method):
    prog = dl.Program(text)
    keep = {k: dev(v) for k, v in rels.items()}
    for k, t in keep.items():
        prog.bind(k, t)
    prog.run(method)
    return prog


def _compare(dl, text, rels, n, tag):
    ref, ref_layers = oprog.evaluate(text, rels, n)
    ref_iters = {tuple(h): it for h, it in ref_layers}
    for method in (dl.DL_EVAL_ITERATION, dl.DL_EVAL_MATRIX):
        announce("program", tag, n, method)
        prog = _run(dl, text, rels, n, method)
        for name, want in ref.items():
            got, ones = prog.fetch(name, n=n)
            got = host(got)
            mism = int((got != want).sum())
            assert mism == 0, f"{tag} n={n} method={method} {name}: {mism} entries differ"
            assert ones == int(want.sum())
        layers = prog.layers()
        assert sorted(tuple(l["heads"]) for l in layers) == sorted(tuple(h) for h, _ in ref_layers)
        for l in layers:
            if l["method"] == dl.DL_EVAL_ITERATION:
                assert l["iters"] == ref_iters[tuple(l["heads"])], (tag, l)
        prog.close()
    return layers


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("n", [1, 5, 64, 257, 600])
def test_cases_vs_oracle(dl, name, n):
    text, _, edbs = CASES[name]
    for seed in range(2):
        rels = {e: _rand(n, 2.0 / n if n > 8 else 0.3, 100 * seed + k) for k, e in enumerate(edbs)}
        if name == "sg":
            rels = {"p": dlgen.to_dense(n, dlgen.forest_edges(n, seed))}
        layers = _compare(dl, text, rels, n, f"{name} seed={seed}")
        assert [l["form"] for l in layers] == FORMS[name]


@pytest.mark.parametrize("n", [4, 100, 300])
def test_stratified_negation(dl, n):
    for seed in range(3):
        rels = {"e": _rand(n, 1.5 / n if n > 8 else 0.35, seed), "f": _rand(n, 1.0 / n if n > 8 else 0.3, 9 + seed)}
        _compare(dl, NEG_TEXT, rels, n, f"negation seed={seed}")


@pytest.mark.parametrize("n", [600, 1000])
@pytest.mark.parametrize("name", ["negation", "even_odd", "transposed", "mixed_general", "layers"])
def test_programs_on_the_large_tile_kernel(dl, name, n):
    """The layered programs with every product forced onto the 256 x 256
    direct-to-LDS step kernel (tile configuration 0, the benchmarked one),
    so its addend (running sums) and complement paths are held to the
    layered oracle, not only to the other evaluation method."""
    ctx = dl.Context()
    ctx.set_tuning("i8", n, 0)
    if name == "negation":
        text = NEG_TEXT
        rels = {"e": _rand(n, 1.5 / n, 31), "f": _rand(n, 1.0 / n, 32)}
    else:
        text, _, edbs = CASES[name]
        rels = {e: _rand(n, 2.0 / n, 40 + k) for k, e in enumerate(edbs)}
    ref, ref_layers = oprog.evaluate(text, rels, n)
    ref_iters = {tuple(h): it for h, it in ref_layers}
    keep = {k: dev(v) for k, v in rels.items()}
    for method in (dl.DL_EVAL_ITERATION, dl.DL_EVAL_MATRIX):
        announce("program cfg0", name, n, method)
        prog = dl.Program(text, ctx=ctx)
        for k, t in keep.items():
            prog.bind(k, t)
        ctx.kernel_stats(0, reset=True)
        ctx.set_timing(True)
        prog.run(method)
        ctx.set_timing(False)
        launches, _ = ctx.kernel_stats(0, reset=True)
        for pname, want in ref.items():
            got, ones = prog.fetch(pname, n=n)
            mism = int((host(got) != want).sum())
            assert mism == 0, f"{name} n={n} method={method} {pname}: {mism} entries differ"
            assert ones == int(want.sum())
        for l in prog.layers():
            if l["method"] == dl.DL_EVAL_ITERATION:
                assert l["iters"] == ref_iters[tuple(l["heads"])], (name, l)
        if method == dl.DL_EVAL_ITERATION:
            assert launches > 0  # products ran (on the forced configuration)
        prog.close()
    ctx.close()


def test_negated_eq_and_converse_in_constant_terms(dl):
    text = ("d(X,Y) :- not eq(X,Y).\n"
            "u(X,Y) :- e(Y,X).\n"
            "w(X,Z) :- d(X,Y), e(Z,Y).\n"
            "v(X,Z) :- e(X,Y), not e(Y,Z).\nv(X,Z) :- v(Y,X), e(Y,Z).")
    n = 130
    _compare(dl, text, {"e": _rand(n, 3.0 / n, 4)}, n, "constants")


def test_dense_and_empty_relations(dl):
    n = 70
    for rel in (np.zeros((n, n), np.uint8), np.ones((n, n), np.uint8)):
        for name in ("tc_right", "transposed", "mixed_general"):
            text, _, edbs = CASES[name]
            _compare(dl, text, {e: rel for e in edbs}, n, f"{name} const")


def test_program_errors(dl):
    with pytest.raises(dl.DLError) as ei:
        dl.Program("t(X,Z) :- e(X,Z).\nt(X,Z) :- t(X,Y), t(Y,Z).")
    assert ei.value.status == 5  # not linear
    with pytest.raises(dl.DLError) as ei:
        dl.Program("p(X,Y) :- e(X,Y).\nq(X,Y) :- e(X,Z), not p(Z,Y).\np(X,Y) :- q(X,Y).")
    assert ei.value.status == 5  # not stratified
    with pytest.raises(dl.DLError) as ei:
        dl.Program("p(X,Y) :- e(X,Y), e(Y,X).")
    assert ei.value.status == 5  # not a chain
    with pytest.raises(dl.DLError) as ei:
        dl.Program("p(X,Y) :- e(X,Y)")
    assert ei.value.status == 1  # syntax
    with pytest.raises(dl.DLError) as ei:
        dl.Program("p(X,Y) :- e(X,y).")
    assert ei.value.status == 1
    prog = dl.Program("p(X,Y) :- e(X,Y).\nq(X,Z) :- p(Y,X), f(Y,Z).")
    with pytest.raises(dl.DLError):
        prog.bind("p", dev(np.eye(4, dtype=np.uint8)))  # defined, not given
    prog.bind("e", dev(np.eye(4, dtype=np.uint8)))
    with pytest.raises(dl.DLError):
        prog.bind("f", dev(np.eye(5, dtype=np.uint8)))  # different n
    with pytest.raises(dl.DLError):
        prog.run()  # f unbound
    with pytest.raises(dl.DLError):
        prog.fetch("p", n=4)  # not run yet


def test_config_tc_program_n4096(dl):
    """Closure program at n = 4096 (ER 1/n and 4/n): both methods against the closure oracle."""
    n = 4096
    for p in (1.0 / n, 4.0 / n):
        a = _rand(n, p, 0, loops=False)
        ref, _, iters, _ = oracle.tc_seminaive(a)
        for method in (dl.DL_EVAL_ITERATION, dl.DL_EVAL_MATRIX):
            announce("tc program 4096", p, method)
            prog = _run(dl, CASES["tc_right"][0], {"e": a}, n, method)
            got, ones = prog.fetch("tc", n=n)
            assert int((host(got) != ref).sum()) == 0
            if method == dl.DL_EVAL_ITERATION:
                assert prog.layers()[0]["iters"] == iters
            prog.close()


def test_config_sg_program_n4096(dl):
    n = 4096
    p = dlgen.to_dense(n, dlgen.forest_edges(n, 1))
    ref, _, iters, _ = oracle.sg_seminaive(p)
    for method in (dl.DL_EVAL_ITERATION, dl.DL_EVAL_MATRIX):
        announce("sg program 4096", method)
        prog = _run(dl, CASES["sg"][0], {"p": p}, n, method)
        got, _ = prog.fetch("sg", n=n)
        assert int((host(got) != ref).sum()) == 0
        prog.close()


# ---------------------------------------------------------------- epsilon solvers


@pytest.mark.parametrize("n", [1, 7, 129, 300])
def test_solve_linear_vs_lapack(dl, n):
    for seed in range(2):
        b = _rand(n, 2.0 / n if n > 8 else 0.3, seed)
        c = _rand(n, 1.5 / n if n > 8 else 0.3, 30 + seed)
        eps = dl.dl_eps_bound(dev(b))
        announce("solve_linear", n, seed)
        r, x = dl.dl_solve_linear(dev(b), dev(c), eps, want_x=True)
        ref = oracle.linear_solve(b, c, eps)
        assert np.allclose(host(x), ref, rtol=1e-12, atol=1e-15)
        tcb = oracle.tc_seminaive(b)[0].astype(np.int64)
        want = ((c.astype(np.int64) + tcb @ c.astype(np.int64)) > 0).astype(np.uint8)
        assert np.array_equal(host(r), want)


def test_solve_linear_validation(dl):
    b = _rand(20, 0.2, 1)
    eps = dl.dl_eps_bound(dev(b))
    with pytest.raises(dl.DLError):
        dl.dl_solve_linear(dev(b), dev(b), eps * 1.01)
    with pytest.raises(dl.DLError):
        dl.dl_solve_linear(dev(b), dev(b), 0.0)


def test_solve_two_sided_vs_kron(dl):
    for seed in range(4):
        n = 5 + 2 * seed
        q, b, c = _rand(n, 0.2, seed), _rand(n, 0.3, 20 + seed), _rand(n, 0.3, 40 + seed)
        eps = 1.0 / (1 + int(b.sum(axis=1).max()) * int(c.sum(axis=0).max()))
        announce("two_sided kron", n)
        r, x, dbl = dl.dl_solve_two_sided(dev(q), dev(b), dev(c), eps, want_x=True)
        assert np.allclose(host(x), oracle.two_sided_kron(q, b, c, eps), rtol=1e-12, atol=1e-15)
        model, _ = oprog.evaluate(TWO_SIDED_TEXT, {"q": q, "b": b, "c": c}, n)
        assert np.array_equal(host(r), model["r"])


@pytest.mark.parametrize("n", [60, 300])
def test_solve_two_sided_threshold(dl, n):
    for seed in range(2):
        q, b, c = _rand(n, 1.0 / n, seed), _rand(n, 2.0 / n, 20 + seed), _rand(n, 2.0 / n, 40 + seed)
        eps = 1.0 / (1 + int(b.sum(axis=1).max()) * int(c.sum(axis=0).max()))
        announce("two_sided", n)
        r, _, dbl = dl.dl_solve_two_sided(dev(q), dev(b), dev(c), eps)
        model, _ = oprog.evaluate(TWO_SIDED_TEXT, {"q": q, "b": b, "c": c}, n)
        assert np.array_equal(host(r), model["r"])
    with pytest.raises(dl.DLError):
        dl.dl_solve_two_sided(dev(q), dev(b), dev(c), eps * 1.5)


def test_measure_peak_sane(dl):
    """The measured matrix-core rates are positive and below the datasheet peaks
    (int8 5.0, fp8 5.0, fp4 10.1, bf16 2.5, fp32 0.157, fp64 0.0786 P/s) with
    10% margin for clock boost."""
    caps = {"i8": 5.0e15, "fp8": 5.0e15, "fp4": 10.1e15, "bf16": 2.5e15, "f32": 157.3e12, "f64": 78.6e12}
    for kind, cap in caps.items():
        announce("peak", kind)
        r = dl.dl_measure_peak(kind)
        assert 0.05 * cap < r < 1.1 * cap, (kind, r)


def test_edge_sizes_and_strides(dl):
    """n = 0 and n = 1 for the solvers and programs; strided (ld > n) inputs
    and outputs are read and written correctly (padding columns untouched)."""
    import torch

    z = torch.zeros((0, 0), dtype=torch.uint8, device="cuda")
    r, x = dl.dl_solve_linear(z, z, 0.5, want_x=True)
    assert r.shape == (0, 0)
    r, x, d = dl.dl_solve_two_sided(z, z, z, 0.5)
    assert r.shape == (0, 0) and d == 0
    one = dev(np.ones((1, 1), np.uint8))
    r, x = dl.dl_solve_linear(one, one, 0.5, want_x=True)
    assert host(r)[0, 0] == 1 and abs(host(x)[0, 0] - 1.0) < 1e-15  # x = 0.5 (1 + x)
    n = 150
    b = _rand(n, 2.0 / n, 3)
    c = _rand(n, 2.0 / n, 4)
    big = np.zeros((n, n + 21), np.uint8)
    big[:, :n] = b * 7
    bview = dev(big)[:, :n]
    out_big = torch.full((n, n + 9), 5, dtype=torch.uint8, device="cuda")
    eps = dl.dl_eps_bound(dev(b))
    announce("strided solve_linear")
    dl.dl_solve_linear(bview, dev(c), eps, out=out_big[:, :n])
    tcb = oracle.tc_seminaive(b)[0].astype(np.int64)
    want = ((c.astype(np.int64) + tcb @ c.astype(np.int64)) > 0).astype(np.uint8)
    assert np.array_equal(host(out_big)[:, :n], want)
    assert np.all(host(out_big)[:, n:] == 5)
    announce("strided program")
    prog = dl.Program(CASES["tc_right"][0])
    prog.bind("e", bview)
    prog.run(dl.DL_EVAL_MATRIX)
    o2 = torch.full((n, n + 3), 9, dtype=torch.uint8, device="cuda")
    _, ones = prog.fetch("tc", out=o2[:, :n])
    ref = oracle.tc_seminaive(b)[0]
    assert np.array_equal(host(o2)[:, :n], ref) and ones == int(ref.sum())
    assert np.all(host(o2)[:, n:] == 9)
    prog.close()


def test_program_rerun_and_rebind(dl):
    """A program can be run again after rebinding its relations; results follow."""
    n = 90
    prog = dl.Program(CASES["even_odd"][0])
    for seed in range(3):
        e = _rand(n, 2.0 / n, 50 + seed, loops=False)
        ed = dev(e)
        prog.bind("e", ed)
        for method in (dl.DL_EVAL_MATRIX, dl.DL_EVAL_ITERATION):
            announce("rerun", seed, method)
            prog.run(method)
            want, _ = oprog.evaluate(CASES["even_odd"][0], {"e": e}, n)
            for name in ("odd", "even"):
                assert np.array_equal(host(prog.fetch(name, n=n)[0]), want[name]), (seed, method, name)
    prog.close()
