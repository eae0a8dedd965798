"""Pins for the CPU FP64 oracle: each test checks it against something other
than itself -- hand-worked examples, brute force in pure Python on tiny inputs,
an independent library (scipy's k-d tree), exact integer arithmetic, the
paper's lemmas and claims as per-query invariants, and a closed-form statistic.
"""
import json
import math
import os

import numpy as np
import pytest

import datagen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


def _col(v):
    return np.asarray(v, np.float32).reshape(-1, 1)


# ---------------------------------------------------------------- worked examples

def test_worked_ownership(orc):
    g = _golden()["ownership_1d"]
    ix = orc.rbc_build_exact(_col(g["X"]), g["rep_idx"])
    assert ix["owner"].tolist() == g["owner"]
    assert ix["psi"].tolist() == g["psi"]
    off, ids = ix["list_off"], ix["list_ids"]
    assert [ids[off[r]:off[r + 1]].tolist() for r in range(2)] == g["lists"]


@pytest.mark.parametrize("metric", ["l2", "l1"])
def test_worked_exact_search(orc, metric):
    g = _golden()["exact_search_1d"]
    X = _col(g["X"])
    ix = orc.rbc_build_exact(X, g["rep_idx"], metric)
    for c in g["cases"]:
        idx, dist, ncand, nkept, kept = orc.rbc_search_exact(_col([c["q"]]), X, ix, c["k"], metric,
                                                             return_kept=True)
        assert kept[0].tolist() == c["kept"], c
        assert idx[0].tolist() == c["idx"], c
        np.testing.assert_allclose(dist[0], c["dist"], rtol=1e-6)


@pytest.mark.parametrize("metric", ["l2", "l1"])
def test_worked_approx_search(orc, metric):
    """The approximate variant (bounds divided by 1 + eps) on the hand-worked
    1-D cases: eps = 0.2 prunes the list that holds the true neighbour."""
    g = _golden()["approx_search_1d"]
    X = _col(g["X"])
    ix = orc.rbc_build_exact(X, g["rep_idx"], metric)
    for c in g["cases"]:
        idx, dist, ncand, nkept, kept = orc.rbc_search_approx(_col([c["q"]]), X, ix, c["k"],
                                                              c["eps"], metric, return_kept=True)
        assert kept[0].tolist() == c["kept"], c
        assert idx[0].tolist() == c["idx"], c
        np.testing.assert_allclose(dist[0], c["dist"], rtol=1e-6)


def test_approx_search_properties(orc):
    """eps = 0 is the exact search; the kept lists shrink as eps grows; every
    answer is the exact k-NN of the kept lists, never closer than BF."""
    rng = np.random.default_rng(3)
    X = rng.standard_normal((3000, 8)).astype(np.float32)
    Q = rng.standard_normal((60, 8)).astype(np.float32)
    reps = np.sort(rng.choice(3000, 55, replace=False))
    ix = orc.rbc_build_exact(X, reps, "l2")
    ref = orc.bf_knn(Q, X, 3, "l2")
    e_idx, e_dist, _, _ = orc.rbc_search_exact(Q, X, ix, 3, "l2")
    a_idx, a_dist, _, _ = orc.rbc_search_approx(Q, X, ix, 3, 0.0, "l2")
    assert np.array_equal(a_idx, e_idx) and np.array_equal(a_dist, e_dist)
    prev = None
    for eps in (0.0, 0.1, 0.5, 2.0):
        idx, dist, ncand, nkept, kept = orc.rbc_search_approx(Q, X, ix, 3, eps, "l2",
                                                              return_kept=True)
        if prev is not None:
            assert not (kept & ~prev).any()          # monotone in eps
        prev = kept
        assert (dist >= ref[1] - 1e-12).all()        # never better than brute force
        for i in range(Q.shape[0]):                  # exact k-NN of the kept lists
            rows = np.concatenate([ix["list_ids"][ix["list_off"][r]:ix["list_off"][r + 1]]
                                   for r in np.nonzero(kept[i])[0]])
            sub_i, sub_d = orc.bf_knn(Q[i:i + 1], X[rows], 3, "l2")
            np.testing.assert_allclose(dist[i], sub_d[0], rtol=1e-12)


@pytest.mark.parametrize("metric", ["l2", "l1"])
def test_range_bf_matches_python(orc, metric):
    """Range search against a pure-Python filter with math.fsum distances, on
    small random inputs, including a radius that lands exactly on a distance
    of integer data (the boundary belongs to the range)."""
    import math

    rng = np.random.default_rng(5)
    X = rng.integers(0, 4, (40, 3)).astype(np.float32)
    Q = rng.integers(0, 4, (6, 3)).astype(np.float32)
    for radius in (0.0, 1.0, 2.0, 2.5):
        off, idx, dist = orc.range_bf(Q, X, radius, metric)
        for i, q in enumerate(Q):
            want = []
            for j, x in enumerate(X):
                if metric == "l2":
                    r = math.sqrt(math.fsum((float(a) - float(b)) ** 2 for a, b in zip(q, x)))
                else:
                    r = math.fsum(abs(float(a) - float(b)) for a, b in zip(q, x))
                if r <= radius:
                    want.append((r, j))
            want.sort()
            got = list(zip(dist[off[i]:off[i + 1]].tolist(), idx[off[i]:off[i + 1]].tolist()))
            assert [j for _, j in got] == [j for _, j in want], (radius, i)
            np.testing.assert_allclose([r for r, _ in got], [r for r, _ in want], rtol=1e-15)


def test_worked_psi_zero_boundary(orc):
    """Strict pruning keeps the nearest representative that owns only itself;
    the literal non-strict rule empties the candidate set (planted mistake)."""
    g = _golden()["psi_zero_boundary"]
    X = _col(g["X"])
    ix = orc.rbc_build_exact(X, g["rep_idx"])
    assert ix["psi"].tolist() == g["psi"]
    idx, dist, ncand, nkept, kept = orc.rbc_search_exact(_col([g["q"]]), X, ix, 1,
                                                         return_kept=True)
    assert kept[0].tolist() == g["strict"]["kept"]
    assert idx[0].tolist() == g["strict"]["idx"]
    assert dist[0].tolist() == g["strict"]["dist"]
    idx, dist, ncand, nkept, kept = orc.rbc_search_exact(_col([g["q"]]), X, ix, 1, strict=False,
                                                         return_kept=True)
    assert kept[0].tolist() == g["literal_nonstrict"]["kept"]
    assert ncand[0] == g["literal_nonstrict"]["ncand"]
    assert idx[0, 0] == -1  # the literal rule loses the answer


def test_worked_oneshot(orc):
    g = _golden()["oneshot_1d"]
    X = _col(g["X"])
    ix = orc.rbc_build_oneshot(X, g["rep_idx"], g["s"])
    assert ix["lists"].tolist() == g["lists"]
    assert ix["psi"].tolist() == g["psi"]
    for c in g["cases"]:
        idx, dist, rep = orc.rbc_search_oneshot(_col([c["q"]]), X, ix, 1)
        assert rep[0] == c["rep"] and idx[0].tolist() == c["idx"], c
        np.testing.assert_allclose(dist[0], c["dist"], rtol=1e-6)
        if "rank" in c:
            assert orc.rank(_col([c["q"]]), X, dist[:, 0])[0] == c["rank"]


def test_worked_oneshot_list_tie(orc):
    g = _golden()["oneshot_list_tie"]
    X = _col(g["X"])
    ix = orc.rbc_build_oneshot(X, g["rep_idx"], g["s"])
    assert ix["lists"].tolist() == g["lists"]
    idx, dist, rep = orc.rbc_search_oneshot(_col([g["q"]]), X, ix, 1)
    assert idx[0].tolist() == g["idx"]
    np.testing.assert_allclose(dist[0], g["dist"], rtol=1e-6)


def test_worked_metrics_disagree(orc):
    g = _golden()["metrics_disagree_2d"]
    X = np.asarray(g["X"], np.float32)
    Q = np.asarray([g["q"]], np.float32)
    for metric in ("l2", "l1"):
        idx, dist = orc.bf_knn(Q, X, 1, metric)
        assert idx[0].tolist() == g[metric]["idx"]
        np.testing.assert_allclose(dist[0], g[metric]["dist"], rtol=1e-15)


def test_worked_bf_tie(orc):
    g = _golden()["bf_tie"]
    X = _col(g["X"])
    for key, k in (("k1", 1), ("k2", 2)):
        idx, dist = orc.bf_knn(_col([g["q"]]), X, k)
        assert idx[0].tolist() == g[key]["idx"]
        assert dist[0].tolist() == g[key]["dist"]


# ---------------------------------------------------------------- brute force pins

def _py_knn(Q, X, k, metric):
    """Pure-Python exhaustive search with math.fsum (exactly rounded sums)."""
    out_i, out_d = [], []
    for q in Q.tolist():
        pairs = []
        for j, x in enumerate(X.tolist()):
            if metric == "l1":
                dd = math.fsum(abs(a - b) for a, b in zip(q, x))
            else:
                dd = math.sqrt(math.fsum((a - b) ** 2 for a, b in zip(q, x)))
            pairs.append((dd, j))
        pairs.sort()
        out_i.append([j for _, j in pairs[:k]])
        out_d.append([dd for dd, _ in pairs[:k]])
    return np.array(out_i), np.array(out_d)


def _assert_knn_match(idx, dist, ref_idx, ref_dist, rtol):
    np.testing.assert_allclose(dist, ref_dist, rtol=rtol, atol=0)
    for i in range(idx.shape[0]):
        for j in range(idx.shape[1]):
            if idx[i, j] != ref_idx[i, j]:
                # only allowed inside a tie class
                assert abs(dist[i, j] - ref_dist[i, j]) <= rtol * max(ref_dist[i, j], 1e-300)
                assert idx[i, j] in set(ref_idx[i].tolist()) or j == idx.shape[1] - 1


@pytest.mark.parametrize("metric", ["l2", "l1"])
@pytest.mark.parametrize("d", [1, 2, 3, 7])
def test_bf_equals_python_brute_force(orc, metric, d):
    rng = np.random.default_rng(100 + d)
    for n in (1, 5, 64):
        X = rng.standard_normal((n, d)).astype(np.float32)
        Q = rng.standard_normal((9, d)).astype(np.float32)
        for k in sorted({1, min(3, n), n}):
            idx, dist = orc.bf_knn(Q, X, k, metric)
            ri, rd = _py_knn(Q, X, k, metric)
            assert np.array_equal(idx, ri)
            np.testing.assert_allclose(dist, rd, rtol=1e-13, atol=0)


def test_bf_k_larger_than_n_pads(orc):
    X = np.zeros((2, 3), np.float32)
    idx, dist = orc.bf_knn(X[:1], X, 4)
    assert idx[0].tolist() == [0, 1, -1, -1]
    assert np.isinf(dist[0, 2:]).all()


@pytest.mark.parametrize("metric,p", [("l2", 2), ("l1", 1)])
@pytest.mark.parametrize("d", [3, 8, 16])
def test_bf_equals_kdtree(orc, metric, p, d):
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(7 * d + p)
    X = rng.standard_normal((3000, d)).astype(np.float32)
    Q = rng.standard_normal((200, d)).astype(np.float32)
    tree = cKDTree(X.astype(np.float64))
    for k in (1, 10):
        idx, dist = orc.bf_knn(Q, X, k, metric)
        rd, ri = tree.query(Q.astype(np.float64), k=k, p=p, eps=0)
        rd, ri = rd.reshape(200, k), ri.reshape(200, k)
        _assert_knn_match(idx, dist, ri, rd, rtol=1e-12)


def test_bf_integer_data_exact(orc):
    """On integer data, squared L2 and L1 distances are integers: compare
    against exact int64 arithmetic, including every (distance, id) tie."""
    rng = np.random.default_rng(5)
    X = rng.integers(0, 4, size=(400, 6)).astype(np.float32)  # many exact ties
    Q = rng.integers(0, 4, size=(50, 6)).astype(np.float32)
    Xi, Qi = X.astype(np.int64), Q.astype(np.int64)
    for metric in ("l2", "l1"):
        diff = Qi[:, None, :] - Xi[None, :, :]
        key = (diff ** 2).sum(-1) if metric == "l2" else np.abs(diff).sum(-1)
        order = np.lexsort((np.broadcast_to(np.arange(400), key.shape), key), axis=1)
        for k in (1, 7, 400):
            idx, dist = orc.bf_knn(Q, X, k, metric)
            assert np.array_equal(idx, order[:, :k])
            ref = np.take_along_axis(key, order[:, :k], 1).astype(np.float64)
            ref = np.sqrt(ref) if metric == "l2" else ref
            assert np.array_equal(dist, ref)


@pytest.mark.parametrize("metric", ["l2", "l1"])
def test_metric_axioms(orc, metric):
    rng = np.random.default_rng(11)
    A = rng.standard_normal((500, 13)).astype(np.float32)
    B = rng.standard_normal((500, 13)).astype(np.float32)
    C = rng.standard_normal((500, 13)).astype(np.float32)
    ab, ba = orc.rho_pairs(A, B, metric), orc.rho_pairs(B, A, metric)
    assert (ab >= 0).all()
    assert np.array_equal(ab, ba)  # symmetric bitwise (|a-b| == |b-a| term by term)
    assert (orc.rho_pairs(A, A, metric) == 0).all()
    ac, bc = orc.rho_pairs(A, C, metric), orc.rho_pairs(B, C, metric)
    assert (ac <= ab + bc + 1e-12).all()


# ---------------------------------------------------------------- RBC invariants

def _cases():
    # (workload, n, m, n_r)
    return [("iid16", 3000, 150, 55), ("sub8", 12000, 120, 110), ("zipf128", 4000, 80, 63)]


@pytest.mark.parametrize("metric", ["l2", "l1"])
@pytest.mark.parametrize("case", _cases())
def test_exact_rbc_equals_bf(orc, metric, case):
    """Exact search returns exactly the brute-force answer (Sec. 5.2)."""
    name, n, m, n_r = case
    X, Q = datagen.database(name, n), datagen.queries(name, m)
    reps = datagen.random_reps(n, n_r, seed=n_r)
    ix = orc.rbc_build_exact(X, reps, metric)
    for k in (1, 10):
        bi, bd = orc.bf_knn(Q, X, k, metric)
        ri, rd, ncand, nkept = orc.rbc_search_exact(Q, X, ix, k, metric)
        assert np.array_equal(ri, bi)
        assert np.array_equal(rd, bd)
        assert (ncand <= n).all() and (nkept >= 1).all()


@pytest.mark.parametrize("n_r", [1, 2, 40])
def test_exact_rbc_degenerate_rep_counts(orc, n_r):
    rng = np.random.default_rng(n_r)
    X = rng.standard_normal((40, 4)).astype(np.float32)
    Q = rng.standard_normal((30, 4)).astype(np.float32)
    reps = datagen.random_reps(40, n_r, seed=3)
    ix = orc.rbc_build_exact(X, reps)
    for k in (1, 5, 40):  # k > n_r makes gamma_k infinite: nothing is pruned
        bi, bd = orc.bf_knn(Q, X, k)
        ri, rd, ncand, _ = orc.rbc_search_exact(Q, X, ix, k)
        assert np.array_equal(ri, bi) and np.array_equal(rd, bd)
        if k > n_r:
            assert (ncand == 40).all()


def test_exact_rbc_with_duplicates(orc):
    """Duplicated rows (exact ties everywhere) still give the BF answer."""
    rng = np.random.default_rng(9)
    base = rng.integers(0, 3, size=(60, 3)).astype(np.float32)
    X = np.concatenate([base, base, base])
    Q = rng.integers(0, 3, size=(40, 3)).astype(np.float32)
    reps = datagen.random_reps(180, 12, seed=4)
    for metric in ("l2", "l1"):
        ix = orc.rbc_build_exact(X, reps, metric)
        for k in (1, 4):
            bi, bd = orc.bf_knn(Q, X, k, metric)
            ri, rd, _, _ = orc.rbc_search_exact(Q, X, ix, k, metric)
            assert np.array_equal(ri, bi) and np.array_equal(rd, bd)


def test_lemma1_claim2_sandwich(orc):
    """Per-query invariants: Lemma 1 (owner of the NN within 3 gamma), Claim 2
    (NN within 4 gamma of its owner, within 7 gamma of q) and the sandwich lemma
    B(q,g) in B(r,2g) in B(q,4g) for r = q's nearest representative."""
    X, Q = datagen.database("sub8", 8000), datagen.queries("sub8", 100)
    reps = datagen.random_reps(8000, 90, seed=1)
    ix = orc.rbc_build_exact(X, reps)
    R = X[reps]
    nn, nnd = orc.bf_knn(Q, X, 1)
    rpos, rdist = orc.bf_knn(Q, R, 1)
    gamma = rdist[:, 0]
    tol = 1e-12
    for i in range(Q.shape[0]):
        x = nn[i, 0]
        owner = ix["owner"][x]
        q_owner = orc.rho_pairs(Q[i:i + 1], R[owner:owner + 1])[0]
        x_owner = orc.rho_pairs(X[x:x + 1], R[owner:owner + 1])[0]
        assert q_owner <= 3 * gamma[i] * (1 + tol)          # Lemma 1
        assert x_owner <= 4 * gamma[i] * (1 + tol)          # Claim 2
        assert nnd[i, 0] <= 7 * gamma[i] * (1 + tol)        # Claim 2
        assert nnd[i, 0] <= gamma[i]                        # R is a subset of X
        # sandwich lemma over the whole database
        r = rpos[i, 0]
        d_q = orc.rho_pairs(np.repeat(Q[i:i + 1], X.shape[0], 0), X)
        d_r = orc.rho_pairs(np.repeat(R[r:r + 1], X.shape[0], 0), X)
        g = gamma[i]
        assert (d_r[d_q <= g] <= 2 * g * (1 + tol)).all()
        assert (d_q[d_r <= 2 * g] <= 4 * g * (1 + tol)).all()


def test_oneshot_success_condition_and_full_lists(orc):
    """App. B: if rho(q, r) < psi_r / 2 for the chosen r, one-shot returns the
    true NN.  With s = n every list is the database and one-shot is BF."""
    rng = np.random.default_rng(12)
    X = rng.standard_normal((3000, 2)).astype(np.float32)
    Q = rng.standard_normal((400, 2)).astype(np.float32)
    reps = datagen.random_reps(3000, 60, seed=2)
    ix = orc.rbc_build_oneshot(X, reps, 300)
    idx, dist, rep = orc.rbc_search_oneshot(Q, X, ix, 1)
    bi, bd = orc.bf_knn(Q, X, 1)
    rdist = orc.rho_pairs(Q, X[reps[rep]])
    guaranteed = rdist < ix["psi"][rep] / 2
    assert guaranteed.sum() > 100
    assert np.array_equal(idx[guaranteed], bi[guaranteed])
    # the returned point is never closer than the true NN
    assert (dist[:, 0] >= bd[:, 0]).all()
    full = orc.rbc_build_oneshot(X[:400], [0, 100, 200], 400)
    i2, d2, _ = orc.rbc_search_oneshot(Q[:50], X[:400], full, 3)
    b2, e2 = orc.bf_knn(Q[:50], X[:400], 3)
    assert np.array_equal(i2, b2) and np.array_equal(d2, e2)


def test_oneshot_lists_are_bf_of_representative(orc):
    """Each one-shot list equals the s nearest points to r found by exhaustive
    pure-Python search (ties by id)."""
    rng = np.random.default_rng(4)
    X = rng.integers(0, 5, size=(50, 2)).astype(np.float32)
    reps = np.array([3, 17, 40])
    ix = orc.rbc_build_oneshot(X, reps, 12)
    ref_i, ref_d = _py_knn(X[reps], X, 12, "l2")
    assert np.array_equal(ix["lists"], ref_i)
    np.testing.assert_allclose(ix["psi"], ref_d[:, -1], rtol=1e-15)


def test_claim1_points_closer_than_nearest_rep(orc):
    """Claim 1: the number T of database points strictly closer to q than its
    nearest representative.  For R drawn as n_r distinct points uniformly at
    random, E[T] = (n - n_r) / (n_r + 1) (the paper's n/n_r is the Bernoulli
    sampling form, counting r_q itself).  Checked as a 4-sigma interval over
    many draws of R."""
    n, n_r, m = 2000, 40, 25
    X = datagen.database("iid16", n)
    Q = datagen.queries("iid16", m)
    _, all_d = orc.bf_knn(Q, X, n)  # sorted distances to every point
    Ts = []
    for seed in range(120):
        reps = datagen.random_reps(n, n_r, seed=1000 + seed)
        _, rd = orc.bf_knn(Q, X[reps], 1)
        Ts.append((all_d < rd[:, :1]).sum(1))
    T = np.concatenate(Ts).astype(np.float64)
    expect = (n - n_r) / (n_r + 1)
    se = T.std(ddof=1) / math.sqrt(T.size)
    assert abs(T.mean() - expect) < 4 * se, (T.mean(), expect, se)
