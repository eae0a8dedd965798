"""GPU parity of the exact Random Ball Cover (Sec. 4 build, Sec. 5.2 search)
against the CPU FP64 oracle, through the C ABI."""
import numpy as np
import pytest

import datagen
from knn_check import assert_knn_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rbc():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1103_2635_amd as rbc

    rbc.lib()
    return rbc


def _dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _search(rbc, ix, Q, k, **kw):
    import torch

    stats = rbc.new_stats()
    idx, dist = rbc.rbc_search(ix, _dev(Q), k, stats=stats, **kw)
    torch.cuda.synchronize()
    return idx.cpu().numpy(), dist.cpu().numpy(), stats.cpu().numpy()


@pytest.mark.parametrize("metric", ["l2", "l1"])
def test_build_matches_oracle(rbc, orc, metric):
    """Ownership lists and the radii psi_r equal the oracle's (psi bit for
    bit: both sum the float64 terms in the same order); inside each list the
    rows are ordered by their distance to the representative (ties by id),
    the stored distances agree with float64 ones to 1e-5."""
    X = datagen.database("sub8", 20000)
    reps = datagen.random_reps(20000, 141, seed=5)
    ix = rbc.rbc_build(_dev(X), 141, metric=metric, rep_idx=reps)
    got = ix.export()
    own, srt = ix.export_order()
    ref = orc.rbc_build_exact(X, reps, metric)
    assert np.array_equal(got["rep_idx"], reps)
    assert np.array_equal(got["list_off"], ref["list_off"])
    assert np.array_equal(got["psi"], ref["psi"])
    off = got["list_off"]
    assert srt.all()
    for r in range(141):
        a, b = off[r], off[r + 1]
        ids = got["list_ids"][a:b]
        assert np.array_equal(np.sort(ids), ref["list_ids"][a:b])   # oracle lists are id-ordered
        key = np.lexsort((ids, own[a:b]))
        assert np.array_equal(key, np.arange(b - a)), r             # (own, id) ascending
        rho = orc.rho_pairs(np.repeat(X[reps[r]][None], b - a, 0), X[ids], metric)
        np.testing.assert_allclose(own[a:b], rho, rtol=1e-5, atol=1e-6)
        assert abs(rho.max() - got["psi"][r]) <= 1e-12 * max(1.0, got["psi"][r])
    ix.free()


def test_long_lists_stay_unsorted_and_exact(rbc, orc):
    """A list longer than the in-LDS sort holds (8192 rows) keeps id order,
    is flagged, and the search scans it whole (same answers)."""
    rng = np.random.default_rng(11)
    X = rng.standard_normal((30000, 16)).astype(np.float32)
    X[:12000] *= 0.01                       # a dense blob owned by one representative
    reps = np.array([0, 12000, 15000, 20000, 25000], np.int64)
    ix = rbc.rbc_build(_dev(X), 5, rep_idx=reps)
    own, srt = ix.export_order()
    off = ix.export()["list_off"]
    sizes = np.diff(off)
    assert (sizes > 8192).any()
    assert np.array_equal(srt, sizes <= 8192)
    Q = np.concatenate([X[:100] + 0.001, rng.standard_normal((100, 16)).astype(np.float32)])
    for k in (1, 10):
        idx, dist, st = _search(rbc, ix, Q, k)
        assert_knn_parity(idx, dist, Q, X, k, "l2", orc)
    ix.free()


CASES = [  # (workload, n, m, n_r)
    ("iid16", 10000, 1000, 100),
    ("sub8", 100000, 1000, 316),
    ("zipf128", 20000, 500, 141),
    ("sub12", 30000, 700, 173),
]


@pytest.mark.parametrize("metric", ["l2", "l1"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_exact_search_equals_bf(rbc, orc, metric, case):
    """Exact search returns the brute-force answer, in one pass and in two.
    One pass: the kept lists are a superset of the oracle's (the pruning
    bounds only widen).  Two passes: the nearest list's bound on the k-th
    neighbour distance keeps fewer lists and scores fewer pairs."""
    name, n, m, n_r = case
    X, Q = datagen.database(name, n), datagen.queries(name, m)
    reps = datagen.representatives(name, n, n_r)
    ix = rbc.rbc_build(_dev(X), n_r, metric=metric, rep_idx=reps)
    oix = orc.rbc_build_exact(X, reps, metric)
    for k in (1, 10):
        ref = orc.bf_knn(Q, X, k, metric)
        idx, dist, st = _search(rbc, ix, Q, k, one_pass=True)
        assert_knn_parity(idx, dist, Q, X, k, metric, orc, ref=ref)
        _, _, ncand, nkept = orc.rbc_search_exact(Q, X, oix, k, metric)
        assert st[3] >= nkept.sum() and st[4] >= ncand.sum()
        assert st[4] <= 1.02 * ncand.sum() + 1000, (st[4], ncand.sum())
        idx2, dist2, st2 = _search(rbc, ix, Q, k)
        assert_knn_parity(idx2, dist2, Q, X, k, metric, orc, ref=ref)
        assert st2[3] <= st[3] and st2[2] <= st[2], (st2, st)
        print("%s %s k=%d pairs one-pass %d two-pass %d" % (name, metric, k, st[2], st2[2]))


@pytest.mark.parametrize("metric", ["l2", "l1"])
def test_exact_search_ragged_and_degenerate(rbc, orc, metric):
    rng = np.random.default_rng(21)
    for (n, m, d, n_r) in ((300, 70, 17, 1), (300, 70, 3, 300), (777, 129, 33, 29),
                           (2000, 300, 96, 45), (50, 1, 129, 7)):
        X = rng.standard_normal((n, d)).astype(np.float32)
        Q = rng.standard_normal((m, d)).astype(np.float32)
        reps = datagen.random_reps(n, n_r, seed=n)
        ix = rbc.rbc_build(_dev(X), n_r, metric=metric, rep_idx=reps)
        for k in sorted({1, min(5, n), min(40, n)}):  # k > n_r: nothing may be pruned
            idx, dist, st = _search(rbc, ix, Q, k)
            assert_knn_parity(idx, dist, Q, X, k, metric, orc)


def test_exact_search_duplicates_and_integer_ties(rbc, orc):
    rng = np.random.default_rng(4)
    base = rng.integers(0, 3, size=(400, 6)).astype(np.float32)
    X = np.concatenate([base, base, base])
    Q = rng.integers(0, 3, size=(150, 6)).astype(np.float32)
    reps = datagen.random_reps(1200, 30, seed=8)
    for metric in ("l2", "l1"):
        ix = rbc.rbc_build(_dev(X), 30, metric=metric, rep_idx=reps)
        for k in (1, 4, 12):
            idx, dist, st = _search(rbc, ix, Q, k)
            ref_i, ref_d = orc.bf_knn(Q, X, k, metric)
            assert np.array_equal(idx, ref_i)
            assert_knn_parity(idx, dist, Q, X, k, metric, orc, ref=(ref_i, ref_d))


def test_matrix_path_integer_ties_two_pass_seed(rbc, orc):
    """Matrix-core path (L2, d = 16) on small-integer data with many exactly
    equal distances: the stage-2 shortlists start from the pass-1 bound on
    the c-th neighbour distance, which on such data often equals the k-th.
    The ids must still be those of the FP64 oracle, (distance, id) order."""
    rng = np.random.default_rng(12)
    base = rng.integers(0, 4, size=(1500, 16)).astype(np.float32)
    X = np.concatenate([base, base[:700]])
    Q = rng.integers(0, 4, size=(300, 16)).astype(np.float32)
    reps = datagen.random_reps(X.shape[0], 48, seed=13)
    ix = rbc.rbc_build(_dev(X), 48, rep_idx=reps)
    for k in (1, 5, 10):
        idx, dist, st = _search(rbc, ix, Q, k)
        ref_i, ref_d = orc.bf_knn(Q, X, k, "l2")
        assert np.array_equal(idx, ref_i)
        assert_knn_parity(idx, dist, Q, X, k, "l2", orc, ref=(ref_i, ref_d))


def test_seeded_representatives_and_errors(rbc):
    import torch

    X = _dev(datagen.database("iid16", 5000))
    a = rbc.rbc_build(X, 70, seed=3).export()["rep_idx"]
    b = rbc.rbc_build(X, 70, seed=3).export()["rep_idx"]
    assert np.array_equal(a, b) and len(np.unique(a)) == 70 and (np.diff(a) > 0).all()
    assert a.min() >= 0 and a.max() < 5000
    with pytest.raises(rbc.RbcError) as e:
        rbc.rbc_build(X, 3, rep_idx=np.array([1, 1, 2]))
    assert e.value.status == -1
    with pytest.raises(rbc.RbcError) as e:
        rbc.rbc_build(X, 5001)
    assert e.value.status == -1
    ix = rbc.rbc_build(X, 10, seed=1)
    with pytest.raises(rbc.RbcError) as e:
        rbc.rbc_search(ix, X[:4], 5001)
    assert e.value.status == -1
    idx, dist = rbc.rbc_search(ix, X[:0], 3)
    torch.cuda.synchronize()
    assert idx.shape == (0, 3)


@pytest.mark.parametrize("m", [1024, 1008])
def test_exact_search_query_count_multiple_of_16(rbc, orc, m):
    """Query counts that are multiples of 16 take the 16-bytes-per-lane work
    list; the answer is the brute-force one, and two calls agree bit for bit
    (the grouping of pass 1 has no fixed order inside a group)."""
    X, Q = datagen.database("sub8", 100000), datagen.queries("sub8", m)
    reps = datagen.representatives("sub8", 100000, 316)
    ix = rbc.rbc_build(_dev(X), 316, rep_idx=reps)
    for k in (1, 10):
        idx, dist, st = _search(rbc, ix, Q, k)
        assert_knn_parity(idx, dist, Q, X, k, "l2", orc)
        idx2, dist2, _ = _search(rbc, ix, Q, k)
        assert np.array_equal(idx, idx2) and np.array_equal(dist, dist2)
    ix.free()


def test_exact_search_deterministic(rbc):
    X, Q = datagen.database("sub8", 50000), datagen.queries("sub8", 900)
    ix = rbc.rbc_build(_dev(X), 223, seed=2)
    a = _search(rbc, ix, Q, 10)
    b = _search(rbc, ix, Q, 10)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("metric", ["l2", "l1"])
@pytest.mark.parametrize("k", [1, 10])
def test_headline_full_size_sampled(rbc, orc, metric, k):
    """n=1,000,000 d=64 (8-dim subspace), n_r=1,000, all 10,000 queries in the
    bench's launch configuration; 48 sampled queries checked against the
    oracle's exhaustive search one by one."""
    import torch

    X, Q = datagen.database("sub8"), datagen.queries("sub8")
    reps = datagen.representatives("sub8")
    ix = rbc.rbc_build(_dev(X), 1000, metric=metric, rep_idx=reps)
    idx, dist, st = _search(rbc, ix, Q, k)
    sample = np.random.default_rng(10 + k).choice(Q.shape[0], 48, replace=False)
    assert_knn_parity(idx[sample], dist[sample], Q[sample], X, k, metric, orc)
    print("candidates/query %.0f lists/query %.1f fallbacks %d" % (st[4] / 1e4, st[3] / 1e4, st[0]))


@pytest.mark.parametrize("metric", ["l2", "l1"])
def test_approximate_search(rbc, orc, metric):
    """prune_eps (the approximate variant beside Sec. 5): eps = 0 is the exact
    search; for eps > 0 the GPU keeps a superset of the oracle's lists (its
    margins only widen), so each returned distance lies between brute force
    and the oracle's approximate answer, and the kept-list count covers the
    oracle's."""
    import torch

    X, Q = datagen.database("sub8", 50000), datagen.queries("sub8", 400)
    reps = datagen.representatives("sub8", 50000, 224)
    ix = rbc.rbc_build(_dev(X), 224, metric=metric, rep_idx=reps)
    oix = orc.rbc_build_exact(X, reps, metric)
    bf_i, bf_d = orc.bf_knn(Q, X, 10, metric)
    e_idx, e_dist, _ = _search(rbc, ix, Q, 10)
    z_idx, z_dist, _ = _search(rbc, ix, Q, 10, prune_eps=0.0)
    assert np.array_equal(e_idx, z_idx) and np.array_equal(e_dist, z_dist)
    for eps in (0.25, 1.0):
        idx, dist, st = _search(rbc, ix, Q, 10, prune_eps=eps)
        o_idx, o_dist, o_ncand, o_nkept = orc.rbc_search_approx(Q, X, oix, 10, eps, metric)
        rho = orc.rho_pairs(np.repeat(Q, 10, 0), X[idx.reshape(-1)], metric).reshape(idx.shape)
        np.testing.assert_allclose(dist, rho, rtol=1e-5)                  # true distances
        assert (rho >= bf_d * (1 - 1e-6)).all()
        assert (rho <= o_dist * (1 + 1e-6) + 1e-12).all()
        assert st[3] >= o_nkept.sum()
        recall = np.mean(idx[:, 0] == bf_i[:, 0])
        print("%s eps=%.2f lists %d (oracle %d) recall@1 %.3f" % (metric, eps, st[3],
                                                                o_nkept.sum(), recall))
    with pytest.raises(rbc.RbcError):
        rbc.bf_search(_dev(Q), _dev(X), 1, metric, prune_eps=0.5)
    with pytest.raises(rbc.RbcError):
        _search(rbc, ix, Q, 1, prune_eps=-1.0)
    ix.free()
