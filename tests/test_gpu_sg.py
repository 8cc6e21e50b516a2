"""Same generation on the GPU through the C ABI, bit-exact against the oracle."""
from __future__ import annotations

import numpy as np
import pytest

import dlgen
import oracle
from tests.gpu_util import announce, dev, gpu, host

pytestmark = gpu


@pytest.fixture(scope="module")
def dl():
    import paper_1608_00139_amd as m

    m.load()
    return m


def _check(dl, p, prec, tag):
    n = p.shape[0]
    announce("sg", tag, n, prec)
    s, iters = dl.dl_sg(dev(p), prec=prec)
    ref, ones, it_ref, _ = oracle.sg_seminaive(p)
    got = host(s)
    mism = int((got != ref).sum())
    assert mism == 0, f"{tag} n={n} prec={prec}: {mism} entries differ"
    assert iters == it_ref
    return got


@pytest.mark.parametrize("n", [1, 3, 64, 100, 257, 600])
def test_forest_sizes(dl, n):
    for seed in range(2):
        p = dlgen.to_dense(n, dlgen.forest_edges(n, seed))
        got = _check(dl, p, "i8", f"forest seed={seed}")
        assert np.array_equal(got, oracle.sg_forest_closed_form(dlgen.forest_parents(n, seed)))


def test_reversed_orientation_is_identity(dl):
    n = 300
    p = dlgen.to_dense(n, dlgen.forest_edges(n, 7, child_to_parent=False))
    announce("sg reversed")
    s, iters = dl.dl_sg(dev(p))
    assert np.array_equal(host(s), np.eye(n, dtype=np.uint8)) and iters == 2


@pytest.mark.parametrize("prec", ["i8", "f32", "bf16", "fp8", "fp4"])
def test_precisions_random_relations(dl, prec):
    for n, seed, pe in ((80, 1, 0.03), (333, 2, 0.004)):
        p = dlgen.to_dense(n, dlgen.er_edges(n, pe, seed, self_loops=True))
        _check(dl, p, prec, f"er seed={seed}")


@pytest.mark.parametrize("n", [200, 256])
def test_per_step_parity(dl, n):
    """Iterate k equals the oracle's (n = 256 is unpadded: the output buffer
    doubles as an iterate buffer)."""
    p = dlgen.to_dense(n, dlgen.forest_edges(n, 4))
    _, ones_ref, iters_ref, _ = oracle.sg_seminaive(p)
    for k in range(0, iters_ref + 2):
        announce("sg steps", k)
        res = dl.dl_sg_steps(dev(p), k, prec="i8")
        assert np.array_equal(host(res.R), oracle.sg_seminaive(p, maxsteps=k)[0]), k
        assert res.steps == min(k, iters_ref)
        assert res.ones == list(ones_ref[: res.steps + 1])


def test_config_forest_n4096(dl):
    """Int8 same generation at n = 4096 on random forests, seeds 0..2."""
    n = 4096
    for seed in range(3):
        p = dlgen.to_dense(n, dlgen.forest_edges(n, seed))
        got = _check(dl, p, "i8", f"cfg4096 seed={seed}")
        assert np.array_equal(got, got.T)
    p = dlgen.to_dense(n, dlgen.forest_edges(n, 0))
    _check(dl, p, "fp4", "cfg4096 fp4")


@pytest.mark.parametrize("n", [100, 600, 1024, 1280, 2000, 3000])
def test_symmetric_stream_k_product(dl, n):
    """S' = [I + T P^T] is symmetric: with int8 operands and the direct-to-LDS
    configuration only its upper-triangle tiles are computed, their K slices
    dealt evenly over the workgroups (stream-K), a tile split over several
    workgroups finished by the last of them to arrive, and the lower tiles
    written as mirror images.  At n = 1280 and 2000 tiles are split over two
    or three workgroups; n = 100 and 600 are padded.  Forests and random
    relations with self-loops, whole model and iteration count."""
    for kind, p in (("forest", dlgen.to_dense(n, dlgen.forest_edges(n, 5))),
                    ("er", dlgen.to_dense(n, dlgen.er_edges(n, 1.2 / n, 6, self_loops=True)))):
        ctx = dl.Context(0)
        ctx.set_tuning("i8", n, 0)
        announce("sg stream-k", kind, n)
        s, iters = dl.dl_sg(dev(p), prec="i8", ctx=ctx)
        ref, _, it_ref, _ = oracle.sg_seminaive(p)
        mism = int((host(s) != ref).sum())
        ctx.close()
        assert mism == 0 and iters == it_ref, (kind, n, mism, iters, it_ref)


def test_symmetric_stream_k_per_step(dl):
    """Every iterate of the stream-K same-generation series at n = 1280 (tiles
    split over workgroups; the partial-tile counters must be back at zero after
    each product) equals the oracle's, with the model sizes."""
    n = 1280
    p = dlgen.to_dense(n, dlgen.er_edges(n, 1.0 / n, 8, self_loops=True))
    _, ones_ref, iters_ref, _ = oracle.sg_seminaive(p)
    ctx = dl.Context(0)
    ctx.set_tuning("i8", n, 0)
    for k in range(0, iters_ref + 2):
        announce("sg stream-k steps", k)
        res = dl.dl_sg_steps(dev(p), k, prec="i8", ctx=ctx)
        assert np.array_equal(host(res.R), oracle.sg_seminaive(p, maxsteps=k)[0]), k
        assert res.steps == min(k, iters_ref)
        assert res.ones == list(ones_ref[: res.steps + 1])
    ctx.close()


def test_symmetric_stream_k_n8192(dl):
    """The stream-K S' product at N = 8192 (528 upper-triangle tiles, 132 K
    slices per workgroup, tiles split over two workgroups), a random forest,
    by the size rule's configuration."""
    n = 8192
    p = dlgen.to_dense(n, dlgen.forest_edges(n, 2))
    _check(dl, p, "i8", "stream-k n8192")
