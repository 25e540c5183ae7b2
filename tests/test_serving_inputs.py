"""Host checks of the serving workload's inputs (synth/serving.py): the request mix, the power-law matrices and
the Poisson arrivals follow the recipe they are documented with."""
import numpy as np

import synth
from synth.serving import ROW_CAP


def test_general_sparse_structure():
    n, m = 5000, 30.0
    A = synth.general_sparse(n, m, 123)
    L = np.diff(A.row_ptr)
    rows = np.repeat(np.arange(n), L)
    same = np.diff(rows) == 0
    assert np.all(np.diff(A.col.astype(np.int64))[same] > 0)  # columns strictly ascending in each row
    assert np.all(L >= 2) and L.max() <= ROW_CAP + 1  # diagonal + 1..cap off-diagonals
    diag = A.col == rows
    assert diag.sum() == n
    off = ~diag
    absum = np.bincount(rows[off], weights=np.abs(A.val[off]), minlength=n)
    ratio = A.val[diag] / absum
    assert np.allclose(ratio, ratio[0]) and 1.05 <= ratio[0] <= 2.0  # one rho per matrix
    assert np.all(np.abs(A.val[off]) < 1.0)
    # band: |j - i| <= max(2m, k_i) with k_i the drawn length (at least the kept one, at most the cap); rows
    # that kept fewer than 2m entries lie within 2m
    k = L - 1
    dist = np.abs(A.col[off].astype(np.int64) - rows[off])
    assert dist.max() <= max(int(2 * m), ROW_CAP)
    short = k[rows[off]] < int(2 * m)
    assert np.mean(dist[short] <= int(2 * m)) > 0.99
    # mean off-diagonal length of a Pareto(2.5, m/3), floored: about 0.55 m
    assert 0.4 * m < k.mean() < 0.6 * m
    # seeded: the same call gives the same matrix
    B = synth.general_sparse(n, m, 123)
    assert np.array_equal(A.col, B.col) and np.array_equal(A.val, B.val)


def test_request_stream_mix():
    reqs = synth.request_stream(4000, seed=5)
    new = [r for r in reqs if r.new]
    reuse = [r for r in reqs if not r.new]
    assert abs(len(reuse) / len(reqs) - 0.7) < 0.03
    kinds = [r.kind for r in new]
    assert abs(kinds.count("general") / len(new) - 0.5) < 0.05
    ns = np.array([r.n_target for r in new])
    assert ns.min() >= 1000 and ns.max() <= 1000000
    assert abs(np.median(np.log(ns)) - 0.5 * (np.log(1e3) + np.log(1e6))) < 0.3  # log-uniform
    # a reused id is one of the last 32 new ids at that point
    seen = []
    for r in reqs:
        if r.new:
            seen.append(r.matrix_id)
        else:
            assert r.matrix_id in seen[-32:]
    assert [r.index for r in reqs] == list(range(len(reqs)))


def test_build_matrix_and_partition():
    reqs = synth.request_stream(64, seed=5, n_max=2e5)
    for r in [q for q in reqs if q.new][:6]:
        A, part, p = synth.build_matrix(r)
        assert p == max(1, -(-A.n // 65536))
        assert part.min() == 0 and part.max() == p - 1 and np.all(np.diff(part) >= 0)
        assert 0.5 * r.n_target <= A.n <= 1.5 * r.n_target + 8


def test_arrivals_are_poisson():
    t = synth.arrival_times(20000, 50.0)
    gaps = np.diff(t)
    assert t[0] == 0.0 and np.all(gaps >= 0)
    assert abs(gaps.mean() - 1 / 50.0) < 0.05 / 50.0
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.05  # exponential: coefficient of variation 1
