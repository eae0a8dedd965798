"""Parity rule for k-NN results against the CPU FP64 oracle.

For every query and every rank j:
  * the returned id equals the oracle's id at rank j, or the two ids' float64
    distances differ by less than ``tie_rtol`` relative (a tie class);
  * the returned distance is within ``dist_rtol`` relative of the oracle's
    distance at rank j (exactly 0 where the oracle's is 0);
  * the ids of one query are distinct.
"""
import numpy as np


def assert_knn_parity(idx, dist, Q, X, k, metric, orc, ref=None, tie_rtol=1e-6, dist_rtol=1e-5,
                      id_of_row=None):
    idx = np.asarray(idx.cpu() if hasattr(idx, "cpu") else idx)
    dist = np.asarray(dist.cpu() if hasattr(dist, "cpu") else dist).astype(np.float64)
    m = Q.shape[0]
    assert idx.shape == (m, k) and dist.shape == (m, k)
    ref_i, ref_d = ref if ref is not None else orc.bf_knn(Q, X, k, metric)
    assert (idx >= 0).all() and (idx < X.shape[0]).all(), "ids out of range"
    for i in range(m):
        assert len(set(idx[i].tolist())) == k, "duplicate ids for query %d" % i
    got64 = orc.rho_pairs(np.repeat(Q, k, axis=0), X[idx.reshape(-1)], metric).reshape(m, k)
    tiny = 1e-300
    mism = idx != ref_i
    bad = mism & (np.abs(got64 - ref_d) > tie_rtol * np.maximum(ref_d, tiny))
    if bad.any():
        q, j = np.argwhere(bad)[0]
        raise AssertionError("query %d rank %d: id %d (rho %.17g) vs oracle id %d (rho %.17g)"
                             % (q, j, idx[q, j], got64[q, j], ref_i[q, j], ref_d[q, j]))
    zero = ref_d == 0
    assert (dist[zero] == 0).all(), "non-zero distance where the oracle has 0"
    err = np.abs(dist - ref_d)
    badd = ~zero & (err > dist_rtol * ref_d)
    if badd.any():
        q, j = np.argwhere(badd)[0]
        raise AssertionError("query %d rank %d: dist %.9g vs oracle %.17g (rel %.3g)"
                             % (q, j, dist[q, j], ref_d[q, j], err[q, j] / ref_d[q, j]))
    return float((err[~zero] / ref_d[~zero]).max()) if (~zero).any() else 0.0
