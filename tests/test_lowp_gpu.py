"""GPU parity of the low-precision brute force (BF16 and FP8 e4m3 ranking
tiles, FP32 re-score, FP64 near-ties, certificate): results must equal the
oracle exactly like the FP32 path; the pre-re-score distances are checked
against the quantisation bound and their error against FP64 is reported."""
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


def _run(rbc, Q, X, k, prec):
    import torch

    stats = rbc.new_stats()
    approx = torch.full((Q.shape[0], k), float("nan"), device="cuda")
    idx, dist = rbc.bf_search(_dev(Q), _dev(X), k, "l2", precision=prec, stats=stats,
                              approx_dist=approx)
    torch.cuda.synchronize()
    return idx.cpu().numpy(), dist.cpu().numpy(), approx.cpu().numpy(), stats.cpu().numpy()


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
@pytest.mark.parametrize("case", [("sub16", 60000, 400, 128), ("sub8", 50000, 300, 64),
                                  ("iid16", 10000, 500, 16), ("zipf128", 30000, 200, 128)],
                         ids=["sub16", "sub8", "iid16", "zipf128"])
def test_lowp_bf_exact(rbc, orc, prec, case):
    name, n, m, d = case
    X, Q = datagen.database(name, n), datagen.queries(name, m)
    for k in (1, 10):
        idx, dist, approx, st = _run(rbc, Q, X, k, prec)
        ref = orc.bf_knn(Q, X, k, "l2")
        assert_knn_parity(idx, dist, Q, X, k, "l2", orc, ref=ref)
        # pre-re-score distances: within the quantisation bound of the FP64 distance
        got64 = orc.rho_pairs(np.repeat(Q, k, 0), X[idx.reshape(-1)], "l2").reshape(idx.shape)
        ok = ~np.isnan(approx)
        rel = np.abs(approx[ok] - got64[ok]) / np.maximum(got64[ok], 1e-30)
        bound = {"bf16": 0.05, "fp8": 0.5}[prec]
        assert rel.max() < bound, (prec, rel.max())
        print("%s %s k=%d pre-re-score rel err max %.3g mean %.3g fallbacks %d" % (
            prec, name, k, rel.max(), rel.mean(), st[0]))


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_lowp_ragged_and_errors(rbc, orc, prec):
    rng = np.random.default_rng(31)
    for (n, m, d) in ((700, 130, 17), (2049, 65, 33), (300, 5, 100)):
        X = rng.standard_normal((n, d)).astype(np.float32)
        Q = rng.standard_normal((m, d)).astype(np.float32)
        for k in (1, 7):
            idx, dist, approx, st = _run(rbc, Q, X, k, prec)
            assert_knn_parity(idx, dist, Q, X, k, "l2", orc)
    import torch

    Xd = torch.zeros((10, 200), device="cuda")
    with pytest.raises(rbc.RbcError) as e:
        rbc.bf_search(Xd[:2], Xd, 1, precision=prec)  # d > 128
    assert e.value.status == -4
    with pytest.raises(rbc.RbcError) as e:
        rbc.bf_search(Xd[:2, :16].contiguous(), Xd[:, :16].contiguous(), 1, "l1", precision=prec)
    assert e.value.status == -4


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
@pytest.mark.parametrize("case", [("sub8", 60000, 700, 64, 245), ("iid16", 20000, 300, 16, 141),
                                  ("zipf128", 30000, 260, 128, 173)],
                         ids=["sub8", "iid16", "zipf128"])
def test_lowp_rbc_exact_search(rbc, orc, prec, case):
    """Exact RBC search (Sec. 5.2) with the low-precision stage-2 tile: same
    answers as the oracle's BF(Q, X) and as the FP32 search of the same index."""
    import torch

    name, n, m, d, n_r = case
    X, Q = datagen.database(name, n), datagen.queries(name, m)
    Xd, Qd = _dev(X), _dev(Q)
    ix = rbc.rbc_build(Xd, n_r, seed=5, precisions=(prec,))
    try:
        for k in (1, 10):
            stats = rbc.new_stats()
            idx, dist = rbc.rbc_search(ix, Qd, k, precision=prec, stats=stats)
            i32, d32 = rbc.rbc_search(ix, Qd, k)
            torch.cuda.synchronize()
            idx, dist = idx.cpu().numpy(), dist.cpu().numpy()
            ref = orc.bf_knn(Q, X, k, "l2")
            assert_knn_parity(idx, dist, Q, X, k, "l2", orc, ref=ref)
            np.testing.assert_array_equal(idx, i32.cpu().numpy())
            # the float32 re-score splits each sum over 64 / c lanes, so the
            # two shortlist lengths may round differently (last bit)
            np.testing.assert_allclose(dist, d32.cpu().numpy(), rtol=1e-6, atol=0)
            st = stats.cpu().numpy()
            print("rbc %s %s k=%d fallbacks %d pairs %d" % (prec, name, k, st[0], st[2]))
    finally:
        ix.free()


def test_lowp_rbc_errors(rbc):
    import torch

    X = torch.randn((3000, 32), device="cuda")
    ix = rbc.rbc_build(X, 50, seed=1, precisions=("bf16",))
    try:
        with pytest.raises(rbc.RbcError) as e:   # index holds no fp8 copy
            rbc.rbc_search(ix, X[:10], 1, precision="fp8")
        assert e.value.status == -4
        idx, _ = rbc.rbc_search(ix, X[:10], 1, precision="bf16")
        assert idx[:, 0].cpu().tolist() == list(range(10))
    finally:
        ix.free()
    with pytest.raises(rbc.RbcError) as e:   # one-shot indexes are FP32 only
        rbc.rbc_build(X, 50, mode="oneshot", s=64, seed=1, precisions=("bf16",))
    assert e.value.status == -4
    with pytest.raises(rbc.RbcError) as e:
        rbc.rbc_build(torch.randn((500, 16), device="cuda"), 20, metric="l1", precisions=("fp8",))
    assert e.value.status == -4


@pytest.mark.parametrize("case", [("sub16", 200000, 3000, 128), ("sub8", 100000, 1500, 64),
                                  ("sub16", 5000, 7, 128)], ids=["sub16", "sub8", "tiny"])
def test_fp8_cascade(rbc, orc, case):
    """FP8 queries whose certificate fails are re-ranked by the fp32 tile
    (a launch sized on the device from the failure count) and stay exact."""
    import torch

    name, n, m, d = case
    X, Q = datagen.database(name, n), datagen.queries(name, m)
    for k in (10, 1):
        idx, dist, approx, st = _run(rbc, Q, X, k, "fp8")
        assert_knn_parity(idx, dist, Q, X, k, "l2", orc)
        print("fp8 %s k=%d cascade %d fallback %d" % (name, k, st[rbc.STAT_CASCADE],
                                                      st[rbc.STAT_FALLBACK]))
        if k == 10 and m >= 1000:
            assert st[rbc.STAT_CASCADE] > 0        # the case the cascade exists for
        assert st[rbc.STAT_FALLBACK] <= max(1, st[rbc.STAT_CASCADE] // 100)
    # the same through an index (the cascade runs over the index rows)
    Xd, Qd = _dev(X), _dev(Q)
    ix = rbc.rbc_build(Xd, max(1, int(np.sqrt(n))), seed=3, precisions=("fp8",))
    try:
        stats = rbc.new_stats()
        idx, dist = rbc.rbc_search(ix, Qd, 10, precision="fp8", stats=stats)
        torch.cuda.synchronize()
        assert_knn_parity(idx.cpu().numpy(), dist.cpu().numpy(), Q, X, 10, "l2", orc)
        st = stats.cpu().numpy()
        print("rbc fp8 %s k=10 cascade %d fallback %d" % (name, st[rbc.STAT_CASCADE],
                                                          st[rbc.STAT_FALLBACK]))
    finally:
        ix.free()
