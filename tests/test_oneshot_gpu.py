"""GPU parity of the one-shot Random Ball Cover (Sec. 4 build with lists of
the s nearest points, Sec. 5.1 search) against the CPU FP64 oracle, through
the C ABI.  The reference for a one-shot search is the oracle's one-shot
search with the same representatives and tie rules, not brute force."""
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


def _search(rbc, ix, Q, k):
    import torch

    stats = rbc.new_stats()
    idx, dist = rbc.rbc_search(ix, _dev(Q), k, stats=stats)
    torch.cuda.synchronize()
    return idx.cpu().numpy(), dist.cpu().numpy(), stats.cpu().numpy()


CASES = [  # (workload, n, m, n_r, s)
    ("zipf128", 40000, 600, 63, 300),
    ("sub8", 30000, 500, 55, 700),
    ("iid16", 10000, 400, 100, 100),
]


@pytest.mark.parametrize("metric", ["l2", "l1"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_oneshot_build_and_search(rbc, orc, metric, case):
    name, n, m, n_r, s = case
    X, Q = datagen.database(name, n), datagen.queries(name, m)
    reps = datagen.representatives(name, n, n_r)
    ix = rbc.rbc_build(_dev(X), n_r, mode="oneshot", metric=metric, s=s, rep_idx=reps)
    got = ix.export()
    ref = orc.rbc_build_oneshot(X, reps, s, metric)
    assert np.array_equal(got["list_off"], np.arange(n_r + 1) * s)
    assert np.array_equal(got["list_ids"].reshape(n_r, s), ref["lists"])
    assert np.array_equal(got["psi"], ref["psi"])
    for k in (1, 10):
        idx, dist, st = _search(rbc, ix, Q, k)
        ri, rd, rep = orc.rbc_search_oneshot(Q, X, ref, k, metric)
        if name == "zipf128":
            assert np.array_equal(idx, ri)  # integer data: exact distances
        assert_knn_parity(idx, dist, Q, X, k, metric, orc, ref=(ri, rd))


def test_oneshot_ties_and_edges(rbc, orc):
    """Integer data with duplicates (ties at the s-th place), s = n (one-shot
    equals brute force), n_r = 1, k = s."""
    rng = np.random.default_rng(17)
    base = rng.integers(0, 4, size=(300, 5)).astype(np.float32)
    X = np.concatenate([base, base])
    Q = rng.integers(0, 4, size=(120, 5)).astype(np.float32)
    for n_r, s, ks in ((9, 40, (1, 7, 40)), (1, 600, (1, 10)), (600, 1, (1,))):
        reps = datagen.random_reps(600, n_r, seed=n_r)
        ix = rbc.rbc_build(_dev(X), n_r, mode="oneshot", s=s, rep_idx=reps)
        ref = orc.rbc_build_oneshot(X, reps, s)
        got = ix.export()
        assert np.array_equal(got["list_ids"].reshape(n_r, s), ref["lists"])
        assert np.array_equal(got["psi"], ref["psi"])
        for k in ks:
            idx, dist, st = _search(rbc, ix, Q, k)
            ri, rd, rep = orc.rbc_search_oneshot(Q, X, ref, k)
            assert np.array_equal(idx, ri)
            assert_knn_parity(idx, dist, Q, X, k, "l2", orc, ref=(ri, rd))
    with pytest.raises(rbc.RbcError) as e:
        rbc.rbc_search(ix, _dev(Q), 2)  # k > s
    assert e.value.status == -1


def test_oneshot_full_size_sampled(rbc, orc):
    """n=2,000,000 d=128 Zipf-clustered integer data, n_r=1,414, s=2,000,
    m=20,000 queries in the bench's launch configuration.  The lists of the
    representatives chosen by 40 sampled queries are rebuilt by the oracle
    and must match exactly; the sampled queries' answers must equal the
    oracle's search of those lists."""
    import torch

    X, Q = datagen.database("zipf128"), datagen.queries("zipf128")
    reps = datagen.representatives("zipf128")
    ix = rbc.rbc_build(_dev(X), 1414, mode="oneshot", s=2000, rep_idx=reps)
    idx, dist, st = _search(rbc, ix, Q, 1)
    got = ix.export()
    lists = got["list_ids"].reshape(1414, 2000)
    sample = np.random.default_rng(5).choice(Q.shape[0], 40, replace=False)
    Qs = Q[sample]
    rpos, _ = orc.bf_knn(Qs, X[reps], 1)
    used = np.unique(rpos[:, 0])
    ref = orc.rbc_build_oneshot(X, reps[used], 2000)
    assert np.array_equal(lists[used], ref["lists"])
    assert np.array_equal(got["psi"][used], ref["psi"])
    for j, i in enumerate(sample):
        L = lists[rpos[j, 0]]
        li, ld = orc.bf_knn(Qs[j:j + 1], X[L], 1)
        assert idx[i, 0] == L[li[0, 0]], (i, idx[i, 0], L[li[0, 0]])
        assert abs(dist[i, 0] - ld[0, 0]) <= 1e-5 * ld[0, 0]
    torch.cuda.synchronize()
