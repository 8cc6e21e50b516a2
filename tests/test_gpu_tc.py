"""Transitive closure on the GPU through the C ABI, bit-exact against the oracle.

Every case compares the whole 0/1 model, the iteration count and the
per-step model sizes with the CPU oracle on the same seeded input.
"""
from __future__ import annotations

import numpy as np
import pytest

import dlgen
import oracle
from tests.golden.load import load_sections
from tests.gpu_util import announce, dev, gpu, host

pytestmark = gpu

PRECS = ["i8", "f32", "bf16", "fp8", "fp4"]


@pytest.fixture(scope="module")
def dl():
    import paper_1608_00139_amd as m

    m.load()
    return m


def _check_closure(dl, a, method, prec, tag=""):
    n = a.shape[0]
    announce("tc", tag, n, method, prec)
    r, iters = dl.dl_tc(dev(a), method=method, prec=prec)
    ref, ones, it_ref, _ = oracle.tc_seminaive(a)
    got = host(r)
    assert got.dtype == np.uint8 and got.shape == (n, n)
    mism = int((got != ref).sum())
    assert mism == 0, f"{tag} n={n} method={method} prec={prec}: {mism} entries differ"
    if method == dl.DL_TC_PLAIN:
        assert iters == it_ref
    else:
        _, hist = oracle.bfs(a, want_matrix=False)
        assert iters == oracle.square_schedule_from_hist(hist)[0]
    return got, iters


def test_worked_example_all_methods(dl):
    g = load_sections("worked_example.txt")
    a = g["R1"].astype(np.uint8)
    for method in (dl.DL_TC_PLAIN, dl.DL_TC_SQUARE):
        for prec in PRECS:
            announce("worked example", method, prec)
            r, iters = dl.dl_tc(dev(a), method=method, prec=prec)
            assert np.array_equal(host(r), g["R2_printed"].astype(np.uint8))
            assert iters == 4


@pytest.mark.parametrize("n", [1, 2, 5, 63, 64, 65, 100, 255, 256, 257, 300, 513, 1000])
@pytest.mark.parametrize("method", [0, 1])
def test_random_sizes_int8(dl, n, method):
    for seed, p in ((0, 1.5 / n), (1, 4.0 / n), (2, 0.05)):
        a = dlgen.to_dense(n, dlgen.er_edges(n, min(p, 1.0), seed))
        _check_closure(dl, a, method, "i8", f"er seed={seed} p={p:.4f}")


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("method", [0, 1])
def test_precisions(dl, prec, method):
    for n, seed in ((200, 3), (777, 4)):
        a = dlgen.to_dense(n, dlgen.er_edges(n, 2.0 / n, seed, self_loops=True))
        _check_closure(dl, a, method, prec, f"prec seed={seed}")


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("n", [300, 512])
def test_per_step_parity(dl, method, n):
    """Iterate k of the GPU series equals the oracle's iterate k, with model
    sizes (n = 512 is unpadded: the output buffer doubles as an iterate
    buffer, so unconverged and converged stops both read it back)."""
    a = dlgen.to_dense(n, dlgen.er_edges(n, 1.3 / n, 5))
    if method == dl.DL_TC_PLAIN:
        _, ones_ref, iters_ref, _ = oracle.tc_seminaive(a)
    else:
        _, ones_ref, iters_ref, _ = oracle.tc_square_literal(a)
    for k in range(0, iters_ref + 2):
        announce("steps", method, k)
        res = dl.dl_tc_steps(dev(a), k, method=method, prec="i8")
        if method == dl.DL_TC_PLAIN:
            rk = oracle.tc_seminaive(a, maxsteps=k)[0]
        else:
            rk = oracle.tc_square_literal(a, maxsteps=k)[0]
        assert np.array_equal(host(res.R), rk), k
        assert res.steps == min(k, iters_ref)
        assert res.converged == (k >= iters_ref)
        assert res.ones == list(ones_ref[: res.steps + 1])


def test_special_graphs(dl):
    cases = {
        "empty": np.zeros((50, 50), np.uint8),
        "complete": 1 - np.eye(40, dtype=np.uint8),
        "cycle": np.roll(np.eye(97, dtype=np.uint8), 1, axis=1),
        "path": np.eye(130, k=1, dtype=np.uint8),
        "selfloops": np.eye(20, dtype=np.uint8),
        "full": np.ones((33, 33), np.uint8),
    }
    for name, a in cases.items():
        for method in (0, 1):
            for prec in ("i8", "f32"):
                _check_closure(dl, a, method, prec, name)


def test_input_encoding_and_strides(dl):
    """Any nonzero byte is true; a strided view (ld > n) is read and written correctly."""
    import torch

    n = 120
    a = dlgen.to_dense(n, dlgen.er_edges(n, 3.0 / n, 9))
    noisy = a * np.random.default_rng(0).integers(1, 256, size=a.shape).astype(np.uint8)
    big = np.zeros((n, n + 37), np.uint8)
    big[:, :n] = noisy
    tbig = dev(big)
    view = tbig[:, :n]
    out_big = torch.full((n, n + 11), 7, dtype=torch.uint8, device="cuda")
    out = out_big[:, :n]
    announce("strides")
    dl.dl_tc(view, method=1, prec="i8", out=out)
    ref = oracle.tc_seminaive(a)[0]
    assert np.array_equal(host(out), ref)
    assert np.all(host(out_big)[:, n:] == 7)  # padding columns untouched


def test_zero_size_and_errors(dl):
    import torch

    announce("zero size")
    r, iters = dl.dl_tc(torch.zeros((0, 0), dtype=torch.uint8, device="cuda"))
    assert iters == 1 and r.shape == (0, 0)
    a = dev(np.eye(8, k=1, dtype=np.uint8))
    with pytest.raises(dl.DLError) as ei:
        dl.dl_tc(a, method=5)
    assert ei.value.status == 1
    with pytest.raises(dl.DLError) as ei:
        dl.dl_tc(a, prec=9)
    assert ei.value.status == 1
    with pytest.raises(dl.DLError) as ei:
        dl.dl_tc(a, out=a)  # output aliases the input
    assert ei.value.status == 1


@pytest.mark.parametrize("count", [1, 2, 5])
@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("prec", ["i8", "f32"])
@pytest.mark.parametrize("n", [300, 512])
def test_batch_matches_oracle(dl, count, method, prec, n):
    """dl_tc_batch: every model and iteration count equal to the oracle's,
    with an empty and a complete relation among random ones (n = 512 is
    unpadded: int8 outputs double as iterate buffers while slots are reused)."""
    inputs = []
    for g in range(count):
        if g == 1:
            a = np.zeros((n, n), np.uint8)
        elif g == 3:
            a = np.ones((n, n), np.uint8)
        else:
            a = dlgen.to_dense(n, dlgen.er_edges(n, (1.0 + g) / n, 10 + g))
        inputs.append(a)
    announce("tc batch", count, method, prec, n)
    rs, its = dl.dl_tc_batch([dev(a) for a in inputs], method=method, prec=prec)
    assert len(rs) == count and len(its) == count
    for g, a in enumerate(inputs):
        ref, _, it_ref, _ = oracle.tc_seminaive(a)
        assert np.array_equal(host(rs[g]), ref), f"graph {g}"
        if method == dl.DL_TC_PLAIN:
            assert its[g] == it_ref, f"graph {g}"
        else:
            _, hist = oracle.bfs(a, want_matrix=False)
            assert its[g] == oracle.square_schedule_from_hist(hist)[0], f"graph {g}"


def test_batch_one_slot_budget_and_errors(dl):
    """A workspace budget that holds one fixpoint runs the batch one at a
    time with the same results; zero counts, zero sizes and overlapping
    buffers."""
    import torch

    n = 300
    inputs = [dlgen.to_dense(n, dlgen.er_edges(n, 2.0 / n, s)) for s in range(3)]
    ctx = dl.Context(workspace_budget=3 << 19)  # Np = 512: one fixpoint needs 1.05 MB, two 2.1 MB
    announce("tc batch one slot")
    rs, its = dl.dl_tc_batch([dev(a) for a in inputs], ctx=ctx)
    for g, a in enumerate(inputs):
        assert np.array_equal(host(rs[g]), oracle.tc_seminaive(a)[0])
    assert dl.dl_tc_batch([]) == ([], [])
    z = [torch.zeros((0, 0), dtype=torch.uint8, device="cuda") for _ in range(3)]
    _, its0 = dl.dl_tc_batch(z)
    assert its0 == [1, 1, 1]
    a0, a1 = dev(inputs[0]), dev(inputs[1])
    out = torch.empty_like(a0)
    with pytest.raises(dl.DLError) as ei:
        dl.dl_tc_batch([a0, a1], outs=[out, out])  # two outputs overlap
    assert ei.value.status == 1
    with pytest.raises(dl.DLError) as ei:
        dl.dl_tc_batch([a0, a1], outs=[a1, out])  # an output overlaps another input
    assert ei.value.status == 1
    with pytest.raises(dl.DLError) as ei:
        dl.dl_tc_batch([a0, a1], method=7)
    assert ei.value.status == 1


@pytest.mark.parametrize("prec", PRECS)
def test_forced_tile_configs(dl, prec):
    """Every tile configuration, forced through dl_tune_set, gives the
    oracle's model and count for both methods on sizes that span several
    tiles of each configuration and end in a ragged tile; same generation on
    each configuration too."""
    ctx = dl.Context()
    elem = {"i8": 1.0, "fp8": 1.0, "f32": 4.0, "bf16": 2.0, "fp4": 0.5}[prec]
    sizes = (300, 700, 2000) if prec == "i8" else (300, 700)
    for n in sizes:
        np_ = (n + 255) // 256 * 256
        cfgs = [0, 1, 2] + ([3] if prec == "i8" else []) + ([4] if np_ * elem <= 2048 else [])
        a = dlgen.to_dense(n, dlgen.er_edges(n, 2.0 / n, 5))
        ref, _, it_plain, _ = oracle.tc_seminaive(a)
        _, hist = oracle.bfs(a, want_matrix=False)
        it_sq = oracle.square_schedule_from_hist(hist)[0]
        p = dlgen.to_dense(n, dlgen.forest_edges(n, 6))
        sg_ref, _, sg_it, _ = oracle.sg_seminaive(p)
        for cfg in cfgs:
            ctx.set_tuning(prec, n, cfg)
            for method, it_ref in ((dl.DL_TC_PLAIN, it_plain), (dl.DL_TC_SQUARE, it_sq)):
                announce("forced cfg", prec, n, cfg, method)
                r, it = dl.dl_tc(dev(a), method=method, prec=prec, ctx=ctx)
                assert np.array_equal(host(r), ref), f"n={n} cfg={cfg} method={method}"
                assert it == it_ref
            announce("forced cfg sg", prec, n, cfg)
            sgr, sit = dl.dl_sg(dev(p), prec=prec, ctx=ctx)
            assert np.array_equal(host(sgr), sg_ref), f"sg n={n} cfg={cfg}"
            assert sit == sg_it
    ctx.close()


def test_autotune(dl, tmp_path):
    """dl_tune picks a valid configuration and records it; fixpoints after
    tuning match the oracle; entries survive a save / load round trip into a
    fresh context; bad configurations are rejected."""
    ctx = dl.Context()
    n = 1000
    announce("autotune i8", n)
    cfg, ms = ctx.tune("i8", n)
    assert 0 <= cfg < 5 and ms > 0
    ent = ctx.tuning()
    assert ent == [{"prec": "i8", "np": 1024, "cfg": cfg, "ms": ms}]
    a = dlgen.to_dense(n, dlgen.er_edges(n, 3.0 / n, 9))
    r, _ = dl.dl_tc(dev(a), ctx=ctx)
    assert np.array_equal(host(r), oracle.tc_seminaive(a)[0])
    announce("autotune f32", 512)
    cfg2, _, cand = ctx.tune("f32", 512, candidates=True)
    assert 0 <= cfg2 < 5 and cand[3] == -1.0 and cand[cfg2] > 0  # the 32 x 32 x 32 form is int8 only
    path = str(tmp_path / "tuning.json")
    ctx.save_tuning(path)
    fresh = dl.Context()
    loaded = fresh.load_tuning(path)
    assert {(e["prec"], e["np"], e["cfg"]) for e in loaded} == {("i8", 1024, cfg), ("f32", 512, cfg2)}
    assert {(e["prec"], e["np"], e["cfg"]) for e in fresh.tuning()} == {("i8", 1024, cfg), ("f32", 512, cfg2)}
    with pytest.raises(dl.DLError):
        fresh.set_tuning("f32", 512, 3)  # the 32 x 32 x 32 configuration is int8 only
    with pytest.raises(dl.DLError):
        fresh.set_tuning("i8", 512, 6)  # no such configuration
    with pytest.raises(dl.DLError):
        fresh.set_tuning("i8", 1024, 5)  # the one-launch fixpoint stops at Np = 512
    with pytest.raises(dl.DLError):
        fresh.set_tuning("f32", 1024, 4)  # 4 KB operand rows do not fit the whole-K tile
    fresh.set_tuning("i8", 1000, -1)
    assert [(e["prec"], e["np"]) for e in fresh.tuning()] == [("f32", 512)]
    ctx.close()
    fresh.close()


def test_config_plain_fp32_n512(dl):
    """Plain FP32 iteration, n = 512, ER p = 2/n, seeds 0..2."""
    n = 512
    for seed in range(3):
        a = dlgen.to_dense(n, dlgen.er_edges(n, 2.0 / n, seed))
        _check_closure(dl, a, dl.DL_TC_PLAIN, "f32", f"cfg512 seed={seed}")


@pytest.mark.parametrize("pname,p", [("1/N", 1.0 / 8192), ("4/N", 4.0 / 8192), ("0.01", 0.01)])
def test_config_n8192_int8_square(dl, pname, p):
    """Int8 repeated squaring at n = 8192 on ER graphs, three seeds each."""
    n = 8192
    for seed in range(3):
        a = dlgen.to_dense(n, dlgen.er_edges(n, p, seed))
        _check_closure(dl, a, dl.DL_TC_SQUARE, "i8", f"cfg8192 p={pname} seed={seed}")


def test_config_n8192_batch(dl):
    """The nine n = 8192 ER graphs as one dl_tc_batch call (the launch the
    benchmark times): each model and count equal to the single-call path,
    which the tests above hold to the oracle at this size."""
    import torch

    n = 8192
    inputs = [dlgen.to_dense(n, dlgen.er_edges(n, p, seed))
              for p in (1.0 / n, 4.0 / n, 0.01) for seed in range(3)]
    announce("tc batch n8192 x9")
    devs = [dev(a) for a in inputs]
    rs, its = dl.dl_tc_batch(devs, method=dl.DL_TC_SQUARE, prec="i8")
    for g, d in enumerate(devs):
        r1, it1 = dl.dl_tc(d, method=dl.DL_TC_SQUARE, prec="i8")
        assert its[g] == it1, f"graph {g}"
        assert torch.equal(rs[g], r1), f"graph {g}"
    del rs, devs


@pytest.mark.parametrize("prec", ["fp4", "fp8", "bf16"])
def test_config_n8192_square_variants(dl, prec):
    """The low-precision squaring variants give the same model at n = 8192."""
    n = 8192
    a = dlgen.to_dense(n, dlgen.er_edges(n, 4.0 / n, 1))
    _check_closure(dl, a, dl.DL_TC_SQUARE, prec, f"cfg8192 {prec}")


@pytest.mark.parametrize("pname,p", [("1/N", 1.0 / 8192), ("4/N", 4.0 / 8192), ("0.01", 0.01)])
def test_config_n8192_fp32_plain(dl, pname, p):
    """The plain FP32 baseline at n = 8192 on all nine ER graphs (p = 1/N is
    the longest plain series: 61-84 iterations): model, iteration count and
    final model size equal to the oracle's."""
    n = 8192
    for seed in range(3):
        a = dlgen.to_dense(n, dlgen.er_edges(n, p, seed))
        _check_closure(dl, a, dl.DL_TC_PLAIN, "f32", f"cfg8192 fp32 p={pname} seed={seed}")


@pytest.mark.parametrize("prec", PRECS)
def test_whole_fixpoint_kernel_vs_chunked(dl, prec):
    """The plain series in one launch (tile configuration 5, the default at
    Np <= 512) and the chunked product kernels (configuration 4 set by the
    caller) against the oracle: ragged sizes over one and two 256-blocks,
    strided input and output, per-step model sizes and capped runs."""
    import torch

    for n in (1, 33, 256, 300, 512):
        a = dlgen.to_dense(n, dlgen.er_edges(n, 2.0 / n if n > 2 else 0.5, 70 + n, self_loops=True))
        ref, ones, it_ref, _ = oracle.tc_seminaive(a)
        for cfg in (5, 4):
            ctx = dl.Context()
            ctx.set_tuning(prec, n, cfg)
            announce("whole fixpoint", prec, n, cfg)
            big = torch.zeros((n, n + 19), dtype=torch.uint8, device="cuda")
            big[:, 3:n + 3] = dev(a * np.uint8(5))
            out = torch.full((n, n + 7), 9, dtype=torch.uint8, device="cuda")
            r, iters = dl.dl_tc(big[:, 3:n + 3], method=dl.DL_TC_PLAIN, prec=prec, out=out[:, :n], ctx=ctx)
            assert np.array_equal(host(r), ref), (prec, n, cfg)
            assert iters == it_ref
            assert bool((out[:, n:] == 9).all())  # padding columns of R untouched
            sr = dl.dl_tc_steps(dev(a), method=dl.DL_TC_PLAIN, prec=prec, max_steps=it_ref + 3, ctx=ctx)
            assert sr.steps == it_ref and sr.converged
            assert sr.ones == [int(x) for x in ones]
            for k in (1, 2, max(1, it_ref - 1)):
                sk = dl.dl_tc_steps(dev(a), method=dl.DL_TC_PLAIN, prec=prec, max_steps=k, ctx=ctx)
                want, ones_k, _, conv_k = oracle.tc_seminaive(a, maxsteps=k)
                assert np.array_equal(host(sk.R), want), (prec, n, cfg, k)
                assert sk.steps == min(k, it_ref) and sk.converged == (k >= it_ref)
                assert sk.ones == [int(x) for x in ones_k]
            ctx.close()


def test_whole_fixpoint_kernel_closed_forms(dl):
    """Closed forms on the one-launch kernel: the empty relation (iters 1),
    the complete digraph (iters 3), a directed cycle of 512 constants
    (D = 512, so 513 iterations: the longest series the kernel can see at
    Np = 512) and a path of 300."""
    n = 512
    cyc = np.zeros((n, n), np.uint8)
    cyc[np.arange(n), (np.arange(n) + 1) % n] = 1
    path = np.eye(300, k=1, dtype=np.uint8)
    cases = [(np.zeros((n, n), np.uint8), np.zeros((n, n), np.uint8), 1),
             (1 - np.eye(n, dtype=np.uint8), np.ones((n, n), np.uint8), 3),
             (cyc, np.ones((n, n), np.uint8), n + 1),
             (path, np.triu(np.ones((300, 300), np.uint8), 1), 300)]
    for a, want, it_want in cases:
        for prec in ("f32", "i8"):
            announce("whole fixpoint closed form", a.shape[0], prec, it_want)
            r, iters = dl.dl_tc(dev(a), method=dl.DL_TC_PLAIN, prec=prec)
            assert iters == it_want and np.array_equal(host(r), want)


def test_whole_fixpoint_config_validation(dl):
    ctx = dl.Context()
    ctx.set_tuning("f32", 512, 5)
    ctx.set_tuning("i8", 300, 5)
    with pytest.raises(dl.DLError):
        ctx.set_tuning("f32", 513, 5)  # Np = 768: rows of 3 KB
    with pytest.raises(dl.DLError):
        ctx.set_tuning("i8", 1000, 5)
    # squaring on a context whose entry is 5 falls back to the size rule
    a = dlgen.to_dense(300, dlgen.er_edges(300, 2.0 / 300, 3))
    r, _ = dl.dl_tc(dev(a), method=dl.DL_TC_SQUARE, prec="i8", ctx=ctx)
    assert np.array_equal(host(r), oracle.tc_seminaive(a)[0])
    ctx.close()


def test_tile_configs_sizes(dl):
    """Sizes that select each tile configuration, with ragged tails."""
    for n in (1500, 2100, 4001):
        a = dlgen.to_dense(n, dlgen.er_edges(n, 2.5 / n, n))
        for prec in ("i8", "bf16", "fp4"):
            _check_closure(dl, a, dl.DL_TC_SQUARE, prec, "tiles")


def test_plain_series_past_the_ring(dl):
    """A directed path of 4500 constants: the plain series needs D + 1 = 4500
    iterations, more steps than the 4096-entry ring of model sizes holds, so
    later steps reuse (and first clear) ring entries.  The model has a closed
    form: r(e_i, e_j) iff i < j."""
    n = 4500
    path = np.zeros((n, n), np.uint8)
    path[np.arange(n - 1), np.arange(1, n)] = 1
    announce("plain past the ring", n)
    r, it = dl.dl_tc(dev(path), method=dl.DL_TC_PLAIN, prec="i8")
    assert it == n
    assert np.array_equal(host(r), np.triu(np.ones((n, n), np.uint8), 1))


def test_kernel_timing(dl):
    """Timing on: one timed product per chunk of steps, none for an empty
    relation; the model is the oracle's."""
    ctx = dl.Context()
    n = 600
    path = np.zeros((n, n), np.uint8)
    path[np.arange(n - 1), np.arange(1, n)] = 1  # D = n - 1: 12 squaring iterations
    ctx.set_timing(True)
    for a in (dlgen.to_dense(n, dlgen.er_edges(n, 1.0 / n, 9)), path):
        ref, _, _, _ = oracle.tc_seminaive(a)
        ctx.kernel_stats(0, reset=True)
        announce("timing", n)
        r, it = dl.dl_tc(dev(a), method=dl.DL_TC_SQUARE, prec="i8", ctx=ctx)
        launches, ms = ctx.kernel_stats(0, reset=True)
        assert np.array_equal(host(r), ref)
        # chunks of the squaring schedule start at steps 2, 8, 12, 20, ...;
        # one is enqueued while no repeat has been seen (it starts <= it)
        assert launches == sum(1 for s0 in (2, 8, 12, 20, 36) if s0 <= it) and ms > 0.0
    _, it0 = dl.dl_tc(dev(np.zeros((n, n), np.uint8)), method=dl.DL_TC_SQUARE, prec="i8", ctx=ctx)
    assert it0 == 1 and ctx.kernel_stats(0, reset=True)[0] == 0
    ctx.set_timing(False)
    ctx.close()


def test_persistent_uneven_passes(dl):
    """n = 4300 (Np = 4352, 17 x 17 = 289 tiles of 256): the persistent step
    kernel's workgroups take one or two tiles, the second with its first
    slice fetched during the first's epilogue; both methods, the int8 and
    the operand-format paths, and same generation on the same sizes."""
    n = 4300
    a = dlgen.to_dense(n, dlgen.er_edges(n, 2.5 / n, 43))
    for prec in ("i8", "bf16", "fp8"):
        _check_closure(dl, a, dl.DL_TC_SQUARE, prec, "persistent")
    _check_closure(dl, a, dl.DL_TC_PLAIN, "i8", "persistent")
    p = dlgen.to_dense(n, dlgen.forest_edges(n, 44))
    sg_ref, _, sg_it, _ = oracle.sg_seminaive(p)
    announce("sg persistent", n)
    s, it = dl.dl_sg(dev(p), prec="i8")
    assert np.array_equal(host(s), sg_ref) and it == sg_it


def test_config_chung_lu_n32768(dl):
    """Power-law digraph (Chung-Lu, gamma 2.1, mean out-degree 8), n = 32768:
    int8 repeated squaring on 1 GiB matrices, the whole model compared.
    The squaring count follows from the plain count: D = plain iters - 1."""
    n = 32768
    a = dlgen.to_dense(n, dlgen.chung_lu_edges(n, 0))
    announce("chung-lu 32768")
    r, iters = dl.dl_tc(dev(a), method=dl.DL_TC_SQUARE, prec="i8")
    ref, ones, it_plain, _ = oracle.tc_seminaive(a)
    got = host(r)
    del r
    assert int((got != ref).sum()) == 0
    d = it_plain - 1
    assert iters == (1 if d == 0 else 2 + int(np.ceil(np.log2(d))) if d > 1 else 2)
    assert int(got.sum()) == int(ones[-1])
