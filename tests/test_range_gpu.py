"""GPU parity of the range search over an exact RBC index (the eps-range
extension of the search algorithms, Sec. 5) against the oracle's direct
float64 range search, through the C ABI.

Every query's set of points must be the oracle's exactly (the float64
decision at the radius is the same computation on both sides); distances are
the float32 roundings of the oracle's float64 distances, and each segment is
in ascending (float32 distance, id) order."""
import ctypes

import numpy as np
import pytest

import datagen

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


def _range(rbc, ix, Q, radius):
    import torch

    off, idx, dist = rbc.rbc_range_search(ix, _dev(Q), radius)
    torch.cuda.synchronize()
    return off.cpu().numpy(), idx.cpu().numpy(), dist.cpu().numpy()


def _assert_range_parity(got, ref):
    off_g, idx_g, dist_g = got
    off_o, idx_o, dist_o = ref
    assert np.array_equal(off_g, off_o), np.flatnonzero(np.diff(off_g) != np.diff(off_o))[:10]
    d32 = dist_o.astype(np.float32)
    seg = np.repeat(np.arange(off_o.shape[0] - 1), np.diff(off_o))
    order = np.lexsort((idx_o, d32, seg))    # the oracle's points in (float32 dist, id) order
    assert np.array_equal(idx_g, idx_o[order])
    assert np.array_equal(dist_g, d32[order])


def _radius_for(X, Q, kth, metric):
    """A radius that holds about kth points for a typical query (median over
    a few queries of the kth smallest float64 distance)."""
    Xd = X.astype(np.float64)
    ds = []
    for q in Q[:16].astype(np.float64):
        diff = Xd - q
        r = np.sqrt((diff * diff).sum(1)) if metric == "l2" else np.abs(diff).sum(1)
        ds.append(np.partition(r, kth)[kth])
    return float(np.median(ds))


@pytest.mark.parametrize("metric", ["l2", "l1"])
@pytest.mark.parametrize("name,d", [("sub8", 64), ("iid16", 16), ("sub8", 37)])
def test_range_matches_oracle(rbc, orc, name, d, metric):
    n = 20000 if name == "sub8" else 10000
    X = np.ascontiguousarray(datagen.database(name, n)[:, :d])
    Q = np.ascontiguousarray(datagen.queries(name, 300)[:, :d])
    radius = _radius_for(X, Q, 40, metric)
    ix = rbc.rbc_build(_dev(X), 120, metric=metric, rep_idx=datagen.random_reps(n, 120, seed=7))
    got = _range(rbc, ix, Q, radius)
    ref = orc.range_bf(Q, X, radius, metric)
    assert got[0][-1] > 300          # the radius holds points for most queries
    _assert_range_parity(got, ref)


@pytest.mark.parametrize("metric", ["l2", "l1"])
def test_range_integer_boundary(rbc, orc, metric):
    """Integer data with the radius equal to an attained distance: the points
    at exactly the radius belong to the result (closed ball)."""
    X = datagen.database("zipf128", 20000)
    Q = datagen.queries("zipf128", 200)
    Xd, q0 = X.astype(np.float64), Q[0].astype(np.float64)
    diff = Xd - q0
    r = np.sqrt((diff * diff).sum(1)) if metric == "l2" else np.abs(diff).sum(1)
    radius = float(np.partition(r, 25)[25])
    ix = rbc.rbc_build(_dev(X), 141, metric=metric, rep_idx=datagen.random_reps(20000, 141, seed=3))
    got = _range(rbc, ix, Q, radius)
    ref = orc.range_bf(Q, X, radius, metric)
    _assert_range_parity(got, ref)
    assert np.any(ref[2] == radius)   # some point lies exactly on the sphere


def test_range_zero_radius_duplicates(rbc, orc):
    """Radius 0: a query equal to database rows returns exactly those rows
    (duplicates included); a query equal to none returns nothing."""
    rng = np.random.default_rng(12)
    base = rng.standard_normal((3000, 24)).astype(np.float32)
    X = np.concatenate([base, base[:500], base[:100]])     # rows 0..99 thrice, 100..499 twice
    Q = np.concatenate([base[:50], base[450:520], rng.standard_normal((30, 24)).astype(np.float32)])
    ix = rbc.rbc_build(_dev(X), 60, rep_idx=datagen.random_reps(X.shape[0], 60, seed=1))
    got = _range(rbc, ix, Q, 0.0)
    ref = orc.range_bf(Q, X, 0.0, "l2")
    _assert_range_parity(got, ref)
    cnt = np.diff(got[0])
    assert np.array_equal(cnt[:50], np.full(50, 3))
    assert np.array_equal(cnt[50:100], np.full(50, 2))
    assert np.array_equal(cnt[100:120], np.full(20, 1))
    assert not cnt[120:].any()


def test_range_empty_and_everything(rbc, orc):
    """A radius below every distance gives empty segments; one above every
    distance gives all n points per query (segments longer than the 8192
    that fit the in-LDS sort)."""
    X = datagen.database("sub8", 20000)
    Q = datagen.queries("sub8", 5)
    ix = rbc.rbc_build(_dev(X), 100, rep_idx=datagen.random_reps(20000, 100, seed=2))
    got = _range(rbc, ix, Q, 1e-3)
    assert not got[0].any() and got[1].shape == (0,)
    got = _range(rbc, ix, Q, 1e6)
    ref = orc.range_bf(Q, X, 1e6, "l2")
    assert got[0][-1] == 5 * 20000
    _assert_range_parity(got, ref)


def test_range_no_queries(rbc):
    import torch

    X = datagen.database("iid16", 2000)
    ix = rbc.rbc_build(_dev(X), 20, seed=1)
    off, idx, dist = rbc.rbc_range_search(ix, torch.empty((0, 16), device="cuda"), 1.0)
    assert off.cpu().tolist() == [0] and idx.numel() == 0 and dist.numel() == 0


def test_range_errors(rbc):
    import torch

    X = datagen.database("iid16", 4000)
    Q = _dev(datagen.queries("iid16", 64))
    ix = rbc.rbc_build(_dev(X), 40, seed=1)
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(rbc.RbcError) as e:
            rbc.rbc_range_count(ix, Q, bad)
        assert e.value.status == -1
    one = rbc.rbc_build(_dev(X), 40, mode="oneshot", s=200, seed=1)
    with pytest.raises(rbc.RbcError) as e:
        rbc.rbc_range_count(one, Q, 1.0)
    assert e.value.status == -4
    # offsets of another radius: the fill is bounded by the segments and the
    # mismatch is reported, for a smaller and for a larger radius
    ws = torch.empty(rbc.rbc_range_workspace_size(ix, 64, 16), dtype=torch.uint8, device="cuda")
    for r_count, r_fill in ((2.0, 3.0), (3.0, 2.0)):
        off = rbc.rbc_range_count(ix, Q, r_count, workspace=ws)
        total = int(off[-1].item())
        idx = torch.empty(max(total, 1), dtype=torch.int64, device="cuda")
        dist = torch.empty(max(total, 1), dtype=torch.float32, device="cuda")
        rc = rbc.lib().rbc_range_search(ix.handle, Q.data_ptr(), 64, 16, ctypes.c_double(r_fill),
                                        off.data_ptr(), idx.data_ptr(), dist.data_ptr(),
                                        ws.data_ptr(), ws.numel(), None)
        assert rc == -1
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    off = torch.empty(65, dtype=torch.int64, device="cuda")
    rc = rbc.lib().rbc_range_count(ix.handle, Q.data_ptr(), 64, 16, ctypes.c_double(1.0),
                                   off.data_ptr(), small.data_ptr(), small.numel(), None)
    assert rc == -5


@pytest.mark.parametrize("metric", ["l2", "l1"])
def test_range_full_size_sampled(rbc, orc, metric):
    """n=1,000,000 d=64 (8-dim subspace), n_r=1,000, all 10,000 queries at a
    radius that holds about 20 points per query (the range line of the
    bench); 32 sampled queries checked against the oracle's direct range
    search one by one."""
    X, Q = datagen.database("sub8"), datagen.queries("sub8")
    reps = datagen.representatives("sub8")
    _, d20 = orc.bf_knn(Q[:8], X, 20, metric)
    radius = float(np.median(d20[:, -1]))
    ix = rbc.rbc_build(_dev(X), 1000, metric=metric, rep_idx=reps)
    off, idx, dist = _range(rbc, ix, Q, radius)
    sample = np.sort(np.random.default_rng(31).choice(Q.shape[0], 32, replace=False))
    r_off, r_idx, r_dist = orc.range_bf(Q[sample], X, radius, metric)
    g_off = np.concatenate([[0], np.cumsum(off[sample + 1] - off[sample])])
    g_idx = np.concatenate([idx[off[i]:off[i + 1]] for i in sample])
    g_dist = np.concatenate([dist[off[i]:off[i + 1]] for i in sample])
    _assert_range_parity((g_off, g_idx, g_dist), (r_off, r_idx, r_dist))
    assert off[-1] > 10 * Q.shape[0]
