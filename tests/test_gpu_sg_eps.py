"""Same-generation epsilon form on the GPU (fp64 Smith doubling).

X = eps (I + P X P^T): values against the vec/Kronecker solve of Sec. 6.3 on
tiny inputs (tolerance 1e-12 relative: every term is non-negative, so the
doubling is componentwise accurate to a few units of roundoff per term),
the residual of the equation at larger n, and the threshold [X > 0] against
the same-generation oracle exactly (zero threshold errors)."""
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


def _eps_max(p):
    d = int(p.sum(axis=1).max()) if p.size else 0
    return 1.0 / (1 + d * d)


@pytest.mark.parametrize("seed", range(4))
def test_values_vs_kronecker(dl, seed):
    n = 6 + 3 * seed
    p = dlgen.to_dense(n, dlgen.er_edges(n, 0.15, seed, self_loops=True))
    eps = _eps_max(p)
    announce("sg eps kron", n, seed)
    s, x, dbl = dl.dl_sg_eps(dev(p), eps, want_x=True)
    ref = oracle.sg_eps_kron(p, eps)
    assert np.allclose(host(x), ref, rtol=1e-12, atol=1e-15)
    assert np.array_equal(host(s), oracle.sg_seminaive(p)[0])


@pytest.mark.parametrize("n", [1, 50, 129, 700])
def test_forest_threshold_and_residual(dl, n):
    for seed in range(2):
        p = dlgen.to_dense(n, dlgen.forest_edges(n, seed))
        eps = _eps_max(p)
        announce("sg eps forest", n, seed)
        s, x, dbl = dl.dl_sg_eps(dev(p), eps, want_x=True)
        xs = host(x)
        assert np.array_equal(host(s), oracle.sg_seminaive(p)[0])
        pf = p.astype(np.float64)
        assert np.allclose(xs, eps * (np.eye(n) + pf @ xs @ pf.T), rtol=1e-12, atol=1e-15)
        assert np.allclose(xs, xs.T, rtol=0, atol=1e-15)


def test_random_relations_threshold(dl):
    for n, seed, pe in ((200, 1, 0.01), (333, 2, 0.004)):
        p = dlgen.to_dense(n, dlgen.er_edges(n, pe, seed, self_loops=True))
        announce("sg eps random", n)
        s, _, _ = dl.dl_sg_eps(dev(p), _eps_max(p))
        assert np.array_equal(host(s), oracle.sg_seminaive(p)[0])


def test_eps_validation(dl):
    p = dlgen.to_dense(40, dlgen.er_edges(40, 0.1, 0))
    eps = _eps_max(p)
    with pytest.raises(dl.DLError):
        dl.dl_sg_eps(dev(p), eps * 1.5)
    s, _, _ = dl.dl_sg_eps(dev(p), eps * 0.5)  # a smaller eps gives the same model
    assert np.array_equal(host(s), oracle.sg_seminaive(p)[0])


def test_config_forest_n4096(dl):
    """n = 4096 random forests, seeds 0..2: zero threshold errors."""
    n = 4096
    for seed in range(3):
        p = dlgen.to_dense(n, dlgen.forest_edges(n, seed))
        announce("sg eps 4096", seed)
        s, _, dbl = dl.dl_sg_eps(dev(p), _eps_max(p))
        errors = int((host(s) != oracle.sg_seminaive(p)[0]).sum())
        assert errors == 0, f"{errors} threshold errors"
