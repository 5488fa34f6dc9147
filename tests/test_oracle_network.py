"""Pins of the oracle's network generator (Sec. 2.1, generator of Sec. 6.1).

The paper's networks are not published, so the generator is pinned by brute
force and by independent re-derivations: a different intersection test
(orientation signs), a different closest-approach computation, clipped lengths,
degrees, connectivity and the merge distance.
"""
import numpy as np
import pytest
from scipy.spatial import cKDTree

from paper_2207_07488_amd import workloads as W


def _clip_interval(a, b):
    """Parameter interval of a + t(b-a), t in [0,1], inside the unit box."""
    lo, hi = 0.0, 1.0
    for k in range(len(a)):
        d = b[k] - a[k]
        if d == 0.0:
            if a[k] < 0 or a[k] > 1:
                return None
            continue
        t1, t2 = (0 - a[k]) / d, (1 - a[k]) / d
        lo, hi = max(lo, min(t1, t2)), min(hi, max(t1, t2))
    return (lo, hi) if lo < hi else None


def _orient(p, q, r):
    return (q[0] - p[0]) * (r[1] - p[1]) - (q[1] - p[1]) * (r[0] - p[0])


def _segments_cross(p1, p2, q1, q2):
    d1, d2 = _orient(q1, q2, p1), _orient(q1, q2, p2)
    d3, d4 = _orient(p1, p2, q1), _orient(p1, p2, q2)
    return (d1 * d2 < 0) and (d3 * d4 < 0)


def _closest_dist(p1, p2, q1, q2):
    """Closest distance of two 3D segments: minimum over the interior stationary
    point and the four edges of the parameter square (independent of the
    oracle's clamped formulation)."""
    d1, d2, r = p2 - p1, q2 - q1, p1 - q1
    best = np.inf

    def dist(s, t):
        return np.linalg.norm(p1 + s * d1 - (q1 + t * d2))

    A = np.array([[d1 @ d1, -(d1 @ d2)], [-(d1 @ d2), d2 @ d2]])
    rhs = np.array([-(d1 @ r), d2 @ r])
    if abs(np.linalg.det(A)) > 1e-300:
        s, t = np.linalg.solve(A, rhs)
        if 0 <= s <= 1 and 0 <= t <= 1:
            best = dist(s, t)
    for s in (0.0, 1.0):
        t = np.clip(((p1 + s * d1 - q1) @ d2) / (d2 @ d2), 0, 1)
        best = min(best, dist(s, t))
    for t in (0.0, 1.0):
        s = np.clip(((q1 + t * d2 - p1) @ d1) / (d1 @ d1), 0, 1)
        best = min(best, dist(s, t))
    return best


def _clipped(seg, dim, tol):
    out = []
    for a, b in zip(seg[:, :dim], seg[:, dim:]):
        iv = _clip_interval(a, b)
        if iv is None:
            continue
        A, B = a + iv[0] * (b - a), a + iv[1] * (b - a)
        if np.linalg.norm(B - A) >= tol:
            out.append((A, B))
    return out


@pytest.mark.parametrize("seed", [1, 2])
def test_grid_search_equals_brute_force_2d(orc, seed):
    seg = W.fiber_segments(2, 400, 0.15, seed=seed)
    a = orc.Network.from_segments(2, seg, merge_tol=1.5e-5, brute=False)
    b = orc.Network.from_segments(2, seg, merge_tol=1.5e-5, brute=True)
    xa, ea, da = a.arrays()
    xb, eb, db = b.arrays()
    assert a.n_raw_nodes == b.n_raw_nodes
    assert np.array_equal(xa, xb) and np.array_equal(ea, eb) and np.array_equal(da, db)


def test_grid_search_equals_brute_force_3d(orc):
    seg = W.fiber_segments(3, 1500, 0.15, seed=5)
    a = orc.Network.from_segments(3, seg, contact_eps=0.01, merge_tol=1.5e-5, dir_lo=4, dir_hi=4, brute=False)
    b = orc.Network.from_segments(3, seg, contact_eps=0.01, merge_tol=1.5e-5, dir_lo=4, dir_hi=4, brute=True)
    assert a.n_raw_nodes == b.n_raw_nodes
    for u, v in zip(a.arrays(), b.arrays()):
        assert np.array_equal(u, v)


def test_crossing_count_matches_orientation_test(orc):
    seg = W.fiber_segments(2, 150, 0.3, seed=11)
    net = orc.Network.from_segments(2, seg, merge_tol=1e-12)
    cl = _clipped(seg, 2, 1e-12)
    assert net.n_segments_kept == len(cl)
    cnt = 0
    for i in range(len(cl)):
        for j in range(i + 1, len(cl)):
            cnt += _segments_cross(cl[i][0], cl[i][1], cl[j][0], cl[j][1])
    assert net.n_raw_nodes - 2 * net.n_segments_kept == cnt


def test_contact_count_matches_closest_distance(orc):
    eps = 0.03
    seg = W.fiber_segments(3, 120, 0.3, seed=3)
    net = orc.Network.from_segments(3, seg, contact_eps=eps, merge_tol=1e-12, dir_lo=4, dir_hi=4)
    cl = _clipped(seg, 3, 1e-12)
    cnt = 0
    for i in range(len(cl)):
        for j in range(i + 1, len(cl)):
            d = _closest_dist(cl[i][0], cl[i][1], cl[j][0], cl[j][1])
            assert abs(d - eps) > 1e-9  # no pair sits on the threshold
            cnt += d < eps
    assert net.n_raw_nodes - 2 * net.n_segments_kept == cnt


def test_total_length_equals_clipped_length(orc):
    # dense enough that every fiber is in the largest component
    seg = W.fiber_segments(2, 200, 0.5, seed=4)
    net = orc.Network.from_segments(2, seg, merge_tol=1e-12)
    x, e, _ = net.arrays()
    cl = _clipped(seg, 2, 1e-12)
    assert net.n_segments_kept == len(cl)
    total_edges = np.linalg.norm(x[e[:, 1]] - x[e[:, 0]], axis=1).sum()
    # segments of the largest component: their clipped end points survive as nodes
    tree = cKDTree(x)
    kept = [(A, B) for A, B in cl if tree.query(A)[0] <= 1e-12]
    assert len(kept) > 0.95 * len(cl)
    total_clip = sum(np.linalg.norm(B - A) for A, B in kept)
    assert abs(total_edges - total_clip) <= 1e-12 * total_clip


def test_degrees_connectivity_and_merge(orc):
    tol = 2e-5
    seg = W.fiber_segments(2, 300, 0.2, seed=1)
    net = orc.Network.from_segments(2, seg, merge_tol=tol)
    x, e, d = net.arrays()
    n = net.n_nodes
    # nodes inside the box, edges valid, no self loops
    assert x.min() >= 0.0 and x.max() <= 1.0
    assert e.min() >= 0 and e.max() < n and np.all(e[:, 0] != e[:, 1])
    # connected (BFS)
    adj = [[] for _ in range(n)]
    for u, v in e:
        adj[u].append(v)
        adj[v].append(u)
    seen = np.zeros(n, bool)
    stack = [0]
    seen[0] = True
    while stack:
        u = stack.pop()
        for v in adj[u]:
            if not seen[v]:
                seen[v] = True
                stack.append(v)
    assert seen.all()
    # no two surviving nodes closer than the merge distance
    assert len(cKDTree(x).query_pairs(tol * (1 - 1e-12))) == 0
    # generic 2D crossings have degree 4, fiber ends degree 1
    deg = np.bincount(e.ravel(), minlength=n)
    assert set(np.unique(deg)) <= {1, 2, 3, 4, 5, 6}
    assert (deg == 4).sum() > 0.5 * (net.n_raw_nodes - 2 * net.n_segments_kept)
    # Dirichlet set: the band at x = 0 and x = 1
    assert np.array_equal(d.astype(bool), (x[:, 0] <= 1e-3) | (x[:, 0] >= 1 - 1e-3))


def test_crossing_density_buffon(orc):
    """Expected crossings of n segments of length l in the unit square, away
    from the boundary: C(n,2) * 2 l^2 / pi (Buffon-Laplace); clipping only
    lowers it, by roughly the fraction of length lost at the boundary."""
    n, l = 2000, 0.05
    seg = W.fiber_segments(2, n, l, seed=9)
    net = orc.Network.from_segments(2, seg, merge_tol=W.merge_tol(l))
    ncr = net.n_raw_nodes - 2 * net.n_segments_kept
    expect = n * (n - 1) / 2 * 2 * l * l / np.pi
    assert 0.85 * expect < ncr < 1.05 * expect


def test_workload_streams():
    # SplitMix64 published first outputs for seed 0
    z = W.splitmix64(0, 0, 3)
    assert [int(v) for v in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    # scalar re-derivation of the counter form for another seed
    M = (1 << 64) - 1

    def mix(x):
        x = ((x ^ (x >> 30)) * 0xBF58476D1CE4E5B9) & M
        x = ((x ^ (x >> 27)) * 0x94D049BB133111EB) & M
        return x ^ (x >> 31)

    seed = 123456789
    z = W.splitmix64(seed, 5, 4)
    assert [int(v) for v in z] == [mix((seed + (i + 1) * 0x9E3779B97F4A7C15) & M) for i in range(5, 9)]
    d = W.unit_directions(3, 1000, 7)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-15)
    # uniform on the sphere: mean ~ 0, second moments ~ 1/3
    assert np.all(np.abs(d.mean(0)) < 0.08) and np.allclose((d ** 2).mean(0), 1 / 3, atol=0.05)
