"""The tile autotuner and the 32x32x2 matrix-core tile shape: results of
bf_search and of the exact RBC search are the oracle's under every pinned
tile choice (shape, stage-2 workgroup count), and after tuning."""
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
    rbc.autotune_clear()
    yield rbc
    rbc.autotune_clear()


def _dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _shortlist(k):
    c = 4
    while c < k + 3:
        c *= 2
    return c


@pytest.mark.parametrize("shape", [16, 32])
@pytest.mark.parametrize("n,m,d", [(4099, 300, 64), (3001, 129, 128), (2500, 70, 17),
                                   (1000, 257, 100)])
@pytest.mark.parametrize("k", [1, 10])
def test_bf_pinned_shape(rbc, orc, shape, n, m, d, k):
    """Ragged rows, queries and features (several 32-row blocks, a partial
    last block, d not a multiple of 16)."""
    import torch

    rng = np.random.default_rng(n + 7 * m + 31 * d + k)
    X = rng.standard_normal((n, d)).astype(np.float32)
    Q = rng.standard_normal((m, d)).astype(np.float32)
    rbc.autotune_set("bf", d, _shortlist(k), shape)
    try:
        idx, dist = rbc.bf_search(_dev(Q), _dev(X), k, "l2")
        torch.cuda.synchronize()
    finally:
        rbc.autotune_clear()
    assert_knn_parity(idx, dist, Q, X, k, "l2", orc)


@pytest.mark.parametrize("shape,blocks,splits,iq", [(16, 1024, 0, 64), (32, 1024, 0, 64),
                                                    (32, 300, 1, 64), (16, 7, 3, 64),
                                                    (16, 1024, 8, 64), (16, 1024, 2, 32),
                                                    (16, 200, 0, 32)])
@pytest.mark.parametrize("k", [1, 10])
def test_search_pinned_shape(rbc, orc, shape, blocks, splits, iq, k):
    """Exact RBC search (two passes) on the small workload under each pinned
    stage-2 configuration, including a persistent grid smaller than the
    device and one that is not a power of two."""
    import torch

    X, Q = datagen.database("iid16"), datagen.queries("iid16")
    reps = datagen.representatives("iid16")
    ix = rbc.rbc_build(_dev(X), len(reps), rep_idx=reps)
    rbc.autotune_set("search", X.shape[1], _shortlist(k), shape, blocks, splits, iq)
    try:
        idx, dist = rbc.rbc_search(ix, _dev(Q), k)
        torch.cuda.synchronize()
    finally:
        rbc.autotune_clear()
        ix.free()
    assert_knn_parity(idx, dist, Q, X, k, "l2", orc)


@pytest.mark.parametrize("shape,iq", [(32, 64), (16, 32)])
def test_search_pinned_shape_headline_sample(rbc, orc, shape, iq):
    """The 10^6 x 64 subspace workload with the 32x32 shape or 32-query items
    pinned for the stage-2 launch: a sample of queries checked against the
    oracle's brute force."""
    import torch

    name = "sub8"
    w = datagen.WORKLOADS[name]
    X = datagen.database(name)
    Q = datagen.queries(name)[:2000]
    reps = datagen.representatives(name)
    ix = rbc.rbc_build(_dev(X), w.n_r, rep_idx=reps)
    rbc.autotune_set("search", X.shape[1], 4, shape, 1024, 0, iq)
    try:
        idx, dist = rbc.rbc_search(ix, _dev(Q), 1)
        torch.cuda.synchronize()
    finally:
        rbc.autotune_clear()
        ix.free()
    sel = np.arange(0, 2000, 40)
    assert_knn_parity(idx.cpu().numpy()[sel], dist.cpu().numpy()[sel], Q[sel], X, 1, "l2", orc)


def test_autotune_search_and_bf(rbc, orc):
    """Tuning picks one of the candidates, reports its time, and later calls
    (which use the choice) still return the oracle's neighbours."""
    import torch

    X, Q = datagen.database("iid16"), datagen.queries("iid16")
    reps = datagen.representatives("iid16")
    Xd, Qd = _dev(X), _dev(Q)
    ix = rbc.rbc_build(Xd, len(reps), rep_idx=reps)
    try:
        r = rbc.autotune_search(ix, Qd, 1)
        assert r["shape"] in (16, 32) and r["blocks"] in (512, 1024, 2048)
        assert r["splits"] in (0, 4) and r["item_queries"] in (32, 64)
        assert r["candidates"] == 18 and r["ms"] > 0 and r["ms_before"] >= r["ms"]
        idx, dist = rbc.rbc_search(ix, Qd, 1)
        b = rbc.autotune_bf(Qd, Xd, 1)
        assert b["shape"] in (16, 32) and b["candidates"] == 2
        bi, bd = rbc.bf_search(Qd, Xd, 1)
        torch.cuda.synchronize()
    finally:
        rbc.autotune_clear()
        ix.free()
    assert_knn_parity(idx, dist, Q, X, 1, "l2", orc)
    assert_knn_parity(bi, bd, Q, X, 1, "l2", orc)


def test_autotune_rejects_untunable(rbc):
    X, Q = datagen.database("iid16"), datagen.queries("iid16")
    with pytest.raises(rbc.RbcError):
        rbc.autotune_bf(_dev(Q), _dev(X), 1, "l1")
