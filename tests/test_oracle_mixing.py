"""Pins of the optimal-mixing distribution reference (Sec. 3).

The estimates are pinned to numpy's mean and biased covariance, the factor to
LAPACK's Cholesky (numpy.linalg.cholesky) and to L L^T = cov, the fallback to
the cases that must trigger it (identical members, fewer members than
variables), the sampler to a hand-worked case and to the first two moments
of many samples, and the variable layout to pinned axes and the
partial-evaluation row order."""
import numpy as np

from oracle import mixing as mx


def population(rs, n, n_points, scale=3.0):
    return (rs.normal(0.0, scale, (n, 2, 3, n_points)) + 20.0).astype(np.float32)


def test_hand_worked_single_variable():
    pts = np.zeros((2, 2, 3, 1), np.float32)
    pts[0, 1, 2, 0] = 1.0
    pts[1, 1, 2, 0] = 3.0
    pinned = np.array([0b011], np.uint8)               # x, y pinned: z in both meshes is free
    dist = mx.estimate(pts, [0, 1], [0], pinned)
    free, mean, L, mode = dist
    assert free == [2, 5] and mode == 1                # mesh-0 z is constant (0): fallback to the diagonal
    assert mean == [0.0, 2.0] and L[1][1] == 1.0 and L[0][0] == 0.0
    z = np.zeros(6, np.float32)
    z[5] = 0.5
    out = mx.sample(dist, z, 4.0, [7, 7, 7, 7, 7, 7])
    assert [float(v) for v in out] == [7, 7, 0, 7, 7, 3.0]   # 2 + sqrt(4) * 0.5, pinned values kept


def test_estimates_match_numpy_and_lapack():
    rs = np.random.default_rng(1)
    pts = population(rs, 60, 10)
    members = list(rs.choice(60, 40, replace=False))
    group = [3, 7]
    free, mean, L, mode = mx.estimate(pts, members, group, None)
    assert mode == 0 and free == list(range(12))
    X = np.stack([[mx.values(pts, i, group, v) for v in free] for i in members])
    np.testing.assert_allclose(mean, X.mean(axis=0), rtol=1e-13)
    cov = np.cov(X, rowvar=False, bias=True)
    L = np.array(L)
    np.testing.assert_allclose(L @ L.T, cov, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(L, np.linalg.cholesky(cov), rtol=1e-9, atol=1e-12)


def test_fallback_cases():
    rs = np.random.default_rng(2)
    pts = population(rs, 30, 6)
    same = np.repeat(pts[:1], 5, axis=0)
    free, mean, L, mode = mx.estimate(same, [0, 1, 2, 3, 4], [1, 4], None)
    assert mode == 1 and np.all(np.array(L) == 0)
    z = rs.normal(size=12).astype(np.float32)
    out = mx.sample((free, mean, L, mode), z, 2.0, [0.0] * 12)
    np.testing.assert_array_equal(np.array(out, np.float32), np.array(mean, np.float32))
    # five distinct members, twelve variables: rank 4, the factor must fail
    free, mean, L, mode = mx.estimate(pts, [0, 1, 2, 3, 4], [1, 4], None)
    assert mode == 1
    X = np.stack([[mx.values(pts, i, [1, 4], v) for v in free] for i in range(5)])
    np.testing.assert_allclose(np.diag(L), np.sqrt(X.var(axis=0)), rtol=1e-12)
    assert np.count_nonzero(np.array(L) - np.diag(np.diag(L))) == 0
    # no members: no distribution
    free, mean, L, mode = mx.estimate(pts, [], [1, 4], None)
    assert mode == 2
    assert np.all(np.isnan(np.array(mx.sample((free, mean, L, mode), z, 1.0, [0.0] * 12), np.float64)))


def test_sample_moments():
    rs = np.random.default_rng(3)
    pts = population(rs, 50, 5)
    group = [0, 2]
    dist = mx.estimate(pts, list(range(50)), group, None)
    free, mean, L, mode = dist
    assert mode == 0
    X = np.stack([[mx.values(pts, i, group, v) for v in free] for i in range(50)])
    cov = np.cov(X, rowvar=False, bias=True)
    n, mult = 12000, 2.25
    Z = rs.normal(size=(n, 12)).astype(np.float32)
    S = np.array([mx.sample(dist, Z[i], mult, [0.0] * 12) for i in range(n)], np.float64)
    sd = np.sqrt(mult * np.diag(cov))
    assert np.all(np.abs(S.mean(axis=0) - np.array(mean)) < 4.5 * sd / np.sqrt(n))
    emp = np.cov(S, rowvar=False)
    scale = np.sqrt(np.outer(np.diag(emp), np.diag(emp)))
    np.testing.assert_allclose(emp / scale, (mult * cov) / (mult * np.sqrt(np.outer(np.diag(cov), np.diag(cov)))),
                               atol=0.05)
    np.testing.assert_allclose(np.diag(emp), mult * np.diag(cov), rtol=0.06)


def test_pinned_axes_and_batch_layout():
    rs = np.random.default_rng(4)
    pts = population(rs, 12, 8)
    pinned = np.zeros(8, np.uint8)
    pinned[5] = 0b101                                   # x and z of point 5 pinned
    grp_off = np.array([0, 2, 4, 7], np.int32)
    grp_pts = np.array([5, 1, 2, 3, 4, 6, 7], np.int32)
    clu_off = np.array([0, 6, 12, 12], np.int32)        # cluster 2 is empty
    clu_members = np.arange(12, dtype=np.int32)
    ep = np.array([0, 3, 9, 2, -1, 4], np.int32)
    eg = np.array([0, 2, 5, 1, 0, 0], np.int32)         # eval 2: group out of range (no rows)
    ec = np.array([0, 1, 0, 2, 1, 7], np.int32)         # eval 3: empty cluster; eval 5: bad cluster
    rows = 2 + 3 + 2 + 2 + 2
    z = rs.normal(size=(rows, 2, 3)).astype(np.float32)
    new = mx.sample_batch(pts, clu_off, clu_members, grp_off, grp_pts, pinned, None, ep, eg, ec, z)
    assert new.shape == (rows, 2, 3)
    # eval 0: group 0 = points (5, 1); point 5 keeps x and z of parent 0 in both meshes
    for m in range(2):
        assert new[0, m, 0] == pts[0, m, 0, 5] and new[0, m, 2] == pts[0, m, 2, 5]
        assert new[0, m, 1] != pts[0, m, 1, 5]
    free = mx.free_variables([5, 1], pinned)
    assert free == [1, 4, 6, 7, 8, 9, 10, 11]
    dist = mx.estimate(pts, list(range(6)), [5, 1], pinned)
    want = mx.sample(dist, z[0:2].reshape(-1), 1.0, [mx.values(pts, 0, [5, 1], v) for v in range(12)])
    np.testing.assert_array_equal(new[0:2].reshape(-1), np.array(want, np.float32))
    assert np.all(np.isfinite(new[2:5]))                # eval 1, cluster 1, group 2 (3 points)
    assert np.all(np.isnan(new[5:7]))                   # eval 3: empty cluster
    assert np.all(np.isnan(new[7:9])) and np.all(np.isnan(new[9:11]))   # bad parent, bad cluster
