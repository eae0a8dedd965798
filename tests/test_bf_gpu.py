"""GPU parity of bf_search (the brute-force primitive, Sec. 3) against the CPU
FP64 oracle, through the C ABI (ctypes binding)."""
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


def _run(rbc, Q, X, k, metric, **kw):
    import torch

    stats = rbc.new_stats()
    idx, dist = rbc.bf_search(_dev(Q), _dev(X), k, metric, stats=stats, **kw)
    torch.cuda.synchronize()
    return idx.cpu().numpy(), dist.cpu().numpy(), stats.cpu().numpy()


@pytest.mark.parametrize("metric", ["l2", "l1"])
@pytest.mark.parametrize("k", [1, 10])
def test_bf_iid16(rbc, orc, metric, k):
    """The small workload: n=10,000, d=16, m=1,000, N(0,1)."""
    X, Q = datagen.database("iid16"), datagen.queries("iid16")
    idx, dist, st = _run(rbc, Q, X, k, metric)
    assert_knn_parity(idx, dist, Q, X, k, metric, orc)


SHAPES = [  # (n, m, d)
    (1, 3, 5), (7, 1, 3), (33, 65, 16), (1000, 257, 17), (4099, 300, 64), (2500, 70, 96),
    (3001, 129, 128), (600, 40, 129), (515, 33, 1), (2000, 100, 8),
]


@pytest.mark.parametrize("metric", ["l2", "l1"])
@pytest.mark.parametrize("shape", SHAPES)
def test_bf_ragged(rbc, orc, metric, shape):
    n, m, d = shape
    rng = np.random.default_rng(n * 31 + m * 7 + d)
    X = rng.standard_normal((n, d)).astype(np.float32)
    Q = rng.standard_normal((m, d)).astype(np.float32)
    for k in sorted({1, min(10, n), min(32, n), n if n <= 64 else 1}):
        idx, dist, st = _run(rbc, Q, X, k, metric)
        assert_knn_parity(idx, dist, Q, X, k, metric, orc)


@pytest.mark.parametrize("metric", ["l2", "l1"])
def test_bf_integer_ties(rbc, orc, metric):
    """Integer data with duplicated rows: exact distance ties everywhere, broken
    by the lower row id."""
    rng = np.random.default_rng(3)
    base = rng.integers(0, 4, size=(700, 24)).astype(np.float32)
    X = np.concatenate([base, base[:300], base[100:400]])
    Q = np.concatenate([base[:50], rng.integers(0, 4, size=(80, 24)).astype(np.float32)])
    for k in (1, 5, 16):
        idx, dist, st = _run(rbc, Q, X, k, metric)
        ref_i, ref_d = orc.bf_knn(Q, X, k, metric)
        # on integer data every distance is exact: ids must match bit for bit
        assert np.array_equal(idx, ref_i)
        assert_knn_parity(idx, dist, Q, X, k, metric, orc, ref=(ref_i, ref_d))


def test_bf_strided_and_large_k(rbc, orc):
    """Row strides wider than d (views of a wider matrix), and k beyond the
    register shortlist (exhaustive float64 path)."""
    import torch

    rng = np.random.default_rng(8)
    Xw = rng.standard_normal((1500, 40)).astype(np.float32)
    Qw = rng.standard_normal((90, 40)).astype(np.float32)
    X, Q = Xw[:, :33], Qw[:, :33]
    Xt, Qt = _dev(Xw)[:, :33], _dev(Qw)[:, :33]
    for k, metric in ((1, "l2"), (12, "l1"), (100, "l2"), (300, "l1")):
        idx, dist = rbc.bf_search(Qt, Xt, k, metric)
        torch.cuda.synchronize()
        assert_knn_parity(idx, dist, Q, X, k, metric, orc)


def test_bf_deterministic(rbc):
    X, Q = datagen.database("sub8", 30000), datagen.queries("sub8", 700)
    a = _run(rbc, Q, X, 10, "l2")
    b = _run(rbc, Q, X, 10, "l2")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_bf_errors(rbc):
    import torch

    X = torch.zeros((10, 4), device="cuda")
    Q = torch.zeros((3, 4), device="cuda")
    with pytest.raises(rbc.RbcError) as e:
        rbc.bf_search(Q, X, 11)
    assert e.value.status == -1
    with pytest.raises(rbc.RbcError) as e:
        rbc.bf_search(Q, X, 0)
    assert e.value.status == -1
    with pytest.raises(rbc.RbcError) as e:   # low precision is L2 only
        rbc.bf_search(Q, X, 1, "l1", precision="bf16")
    assert e.value.status == -4
    idx, dist = rbc.bf_search(Q[:0], X, 2)
    assert idx.shape == (0, 2)


@pytest.mark.parametrize("metric", ["l2", "l1"])
@pytest.mark.parametrize("k", [1, 10])
def test_bf_headline_full_size_sampled(rbc, orc, metric, k):
    """n=1,000,000 d=64 8-dim-subspace workload, all 10,000 queries on the GPU
    in the bench's launch configuration; 64 sampled queries checked against
    the oracle one by one."""
    import torch

    X, Q = datagen.database("sub8"), datagen.queries("sub8")
    stats = rbc.new_stats()
    idx, dist = rbc.bf_search(_dev(Q), _dev(X), k, metric, stats=stats)
    torch.cuda.synchronize()
    idx, dist = idx.cpu().numpy(), dist.cpu().numpy()
    sample = np.random.default_rng(k).choice(Q.shape[0], 64, replace=False)
    assert_knn_parity(idx[sample], dist[sample], Q[sample], X, k, metric, orc)
    print("fallbacks", int(stats[0]), "near-ties", int(stats[1]))
