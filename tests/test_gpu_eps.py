"""The fp64 epsilon solve on the GPU through the C ABI.

The thresholded model must equal the closure oracle exactly (Theorem 1:
zero threshold errors); the real solution X is compared with exact rational
arithmetic on tiny inputs and with an fp64 LAPACK solve elsewhere.

Tolerance for X: the solve is componentwise stable here (every update adds
terms of one sign, see the kernel notes), so each entry carries a relative
error of a few units of roundoff per accumulated term; 1e-12 relative plus
1e-15 absolute (for the LAPACK comparison, whose own partial-pivoting error
is normwise, 1e-13 absolute) covers n up to a few thousand with margin.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np
import pytest

import dlgen
import oracle
from tests.golden.load import load_sections
from tests.gpu_util import announce, dev, gpu, host

pytestmark = gpu


@pytest.fixture(scope="module")
def dl():
    import paper_1608_00139_amd as m

    m.load()
    return m


def test_worked_example_values(dl):
    g = load_sections("worked_example.txt")
    a = g["R1"].astype(np.uint8)
    announce("eps worked example")
    r, x, flag = dl.dl_solve_eps(dev(a), 0.5, want_x=True, underflow=True)
    assert flag == 0
    xs = host(x)
    exact = np.array([[1, 4, 2, 0], [2, 1, 4, 0], [4, 2, 1, 0], [4, 2, 1, 0]]) / 7.0
    assert np.allclose(xs, exact, rtol=1e-14, atol=1e-16)
    assert np.all(np.abs(xs - g["X_printed"]) < 1e-4)
    assert np.array_equal(host(r), g["R2_printed"].astype(np.uint8))
    assert np.all(xs[:, 3] == 0.0)  # exact zeros stay exact


@pytest.mark.parametrize("seed", range(5))
def test_exact_rationals_tiny(dl, seed):
    n = 3 + seed
    a = dlgen.to_dense(n, dlgen.er_edges(n, 0.35, seed, self_loops=True))
    d = int(a.sum(axis=1).max())
    eps = Fraction(1, 1 + d)
    ex = np.array([[float(v) for v in row] for row in oracle.eps_solve_exact(a, eps)])
    announce("eps exact", seed)
    r, x = dl.dl_solve_eps(dev(a), float(eps), want_x=True)
    assert np.allclose(host(x), ex, rtol=1e-12, atol=1e-15)
    assert np.array_equal(host(r), oracle.tc_seminaive(a)[0])


@pytest.mark.parametrize("n", [1, 17, 128, 129, 300, 1000])
def test_random_vs_lapack_and_closure(dl, n):
    for seed, pe in ((0, 2.0 / n), (1, 0.02)):
        a = dlgen.to_dense(n, dlgen.er_edges(n, min(pe, 1.0), seed, self_loops=(seed == 1)))
        eps = oracle.eps_bound(a)
        announce("eps random", n, seed)
        r, x = dl.dl_solve_eps(dev(a), eps, want_x=True)
        xs = host(x)
        ref = oracle.eps_solve(a, eps)
        assert np.allclose(xs, ref, rtol=1e-12, atol=1e-13)
        assert np.all(xs >= 0) and np.all(xs <= 1 + 1e-12)  # Lemma 1
        assert np.array_equal(host(r), oracle.tc_seminaive(a)[0])


def test_underflow_flag_boundary(dl):
    """Directed paths at eps = 1/2: X_ij = 2^-(j-i) exactly.  A path of 1000
    constants keeps every entry at least 2^-999, a normal double far from
    the smallest one (flag 0, model exact); one of 1030 has entries below
    2^-1022 (flag 1; no false positive either way)."""
    for n, want in ((1000, 0), (1030, 1)):
        a = np.eye(n, k=1, dtype=np.uint8)
        ref = np.triu(np.ones((n, n), np.uint8), 1)
        announce("eps underflow flag", n)
        r, x, flag = dl.dl_solve_eps(dev(a), 0.5, want_x=True, underflow=True)
        assert flag == want, (n, flag)
        got = host(r)
        assert not np.any(got & (1 - ref)), "false positive"
        if want == 0:
            assert np.array_equal(got, ref)
            assert host(x)[0, n - 1] == 2.0 ** -(n - 1)


def test_eps_validation(dl):
    a = dlgen.to_dense(50, dlgen.er_edges(50, 0.1, 3))
    bound = oracle.eps_bound(a)
    announce("eps validation")
    assert abs(dl.dl_eps_bound(dev(a)) - bound) < 1e-15
    with pytest.raises(dl.DLError) as ei:
        dl.dl_solve_eps(dev(a), bound * 1.01)
    assert ei.value.status == 1
    with pytest.raises(dl.DLError):
        dl.dl_solve_eps(dev(a), 0.0)
    r, _ = dl.dl_solve_eps(dev(a), bound * 0.25)  # smaller eps is allowed
    assert np.array_equal(host(r), oracle.tc_seminaive(a)[0])


def test_underflow_negative_control(dl):
    """A long directed path: X_ij = eps^(j-i) falls below fp64's range.

    The threshold must show no false positive, be exact for distances whose
    weight is a normal fp64 number, and miss the far pairs: this proves the
    threshold check can fail and bounds where it does.
    """
    n = 1500
    a = np.eye(n, k=1, dtype=np.uint8)
    announce("eps underflow control")
    r, x, flag = dl.dl_solve_eps(dev(a), 0.5, want_x=True, underflow=True)
    assert flag == 1, "the call must report that entries may be lost"
    got = host(r)
    ref = oracle.tc_seminaive(a)[0]
    assert not np.any(got & (1 - ref)), "false positive"
    i, j = np.nonzero(ref)
    dist = j - i
    near = dist <= 1000
    assert np.all(got[i[near], j[near]] == 1)
    assert np.any(got[i[~near], j[~near]] == 0)


@pytest.mark.parametrize("pname,p", [("1/N", 1.0 / 8192), ("4/N", 4.0 / 8192), ("0.01", 0.01)])
def test_config_n8192_zero_threshold_errors(dl, pname, p):
    """n = 8192, eps = 0.5 / (max row sum + 1), all nine ER graphs: the
    thresholded X equals the closure oracle's model (zero threshold errors)
    and the call reports no possible underflow."""
    n = 8192
    for seed in range(3):
        a = dlgen.to_dense(n, dlgen.er_edges(n, p, seed))
        eps = 0.5 / (1.0 + float(a.sum(axis=1).max()))
        announce("eps 8192", pname, seed)
        r, _, flag = dl.dl_solve_eps(dev(a), eps, underflow=True)
        ref = oracle.tc_seminaive(a)[0]
        errors = int((host(r) != ref).sum())
        assert errors == 0, f"p={pname} seed={seed}: {errors} threshold errors"
        assert flag == 0
