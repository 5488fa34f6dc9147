"""Pins of the oracle's network diagnostics (Assumption 3.4, Lemma 3.5; Sec.
6.1 and 6.2.1): closed forms of the box density and of lambda_2 on a path,
the BFS joining of a box subgraph, and the grid row of Table 6.3 (sigma and
mu of the Example 3.7 grid, which the paper prints to one and two digits)."""
import numpy as np
import pytest

from paper_2207_07488_amd import workloads as W
import diagnostics as D  # oracle/diagnostics.py (the oracle directory is on sys.path)


def test_box_density_of_grid():
    """Example 3.7 grid, n = 16, 4 x 4 boxes: an interior box holds 4 x 4 nodes
    of mass 2/n each, so its density is 2 n; the box at the upper corner also
    holds the boundary rows (closed upper faces)."""
    n, nb = 16, 4
    x, e = W.grid_network(n)
    dens, sigma, rho = D.homogeneity(x, e, nb)
    d = dens.reshape(nb, nb)
    assert d[1, 1] == pytest.approx(2 * n, rel=1e-14) and d[2, 2] == pytest.approx(2 * n, rel=1e-14)
    # lower corner: rows/columns 0..3, boundary nodes of mass 1.5/n, corner 1/n
    low = (9 * 2 + 6 * 1.5 + 1.0) / n * nb * nb
    assert d[0, 0] == pytest.approx(low, rel=1e-14)
    # upper corner: 5 x 5 nodes, the outer row and column on the boundary
    up = (16 * 2 + 8 * 1.5 + 1.0) / n * nb * nb
    assert d[3, 3] == pytest.approx(up, rel=1e-14)
    assert sigma == pytest.approx(up / low, rel=1e-14) and rho == pytest.approx(low, rel=1e-14)


@pytest.mark.parametrize("m", [5, 17, 60])
def test_lambda2_of_a_path(m):
    """A straight chain of m nodes, spacing h, weights 1/h, lumped masses h/2
    at the ends: lambda_2 = (2/h^2)(1 - cos(pi/(m-1)))."""
    h = 0.01
    x = np.stack([0.2 + h * np.arange(m), np.full(m, 0.5)], 1)
    e = np.stack([np.arange(m - 1), np.arange(1, m)], 1)
    lam = D.lambda2(x, e, list(range(m - 1)))
    assert lam == pytest.approx(2 / h ** 2 * (1 - np.cos(np.pi / (m - 1))), rel=1e-9)


def test_box_subgraph_is_joined_outside_the_box():
    """Two edges in the box [0.25, 0.5]^2 whose pieces leave it and meet only
    through a node 0.06 outside: BFS adds the two edges to that node when it is
    within r0, and the box fails (None) when it is not."""
    x = np.array([[0.30, 0.30], [0.45, 0.30], [0.30, 0.45], [0.45, 0.45], [0.52, 0.30], [0.52, 0.45],
                  [0.56, 0.375]])
    e = np.array([[0, 1], [2, 3], [1, 4], [3, 5], [4, 6], [5, 6]])
    import collections
    adj = collections.defaultdict(list)
    for k, (u, v) in enumerate(e):
        adj[int(u)].append((int(v), k))
        adj[int(v)].append((int(u), k))
    cand = np.arange(len(x))
    b = 1 + 4 * 1  # box (1, 1) of a 4 x 4 split
    assert sorted(D.box_subgraph(x, e, adj, b, 4, 0.1, cand)) == [0, 1, 2, 3, 4, 5]
    assert D.box_subgraph(x, e, adj, b, 4, 0.03, cand) is None


@pytest.mark.slow
def test_table_6_3_grid_row():
    """Table 6.3 (Sec. 6.2.1): sigma (1.0, 1.0, 1.1, 1.1) and mu (0.45, 0.47,
    0.48, 0.51) of the (2^9 + 1)^2 grid for H^-1 = 4, 8, 16, 32; sigma to its
    printed digit, mu to 0.01."""
    x, e = W.grid_network(512)
    printed = {4: (1.0, 0.45), 8: (1.0, 0.47), 16: (1.1, 0.48), 32: (1.1, 0.51)}
    for nb, (s_p, m_p) in printed.items():
        _, sigma, _ = D.homogeneity(x, e, nb)
        _, mu = D.connectivity(x, e, nb)
        assert round(sigma, 1) == s_p, (nb, sigma)
        assert abs(mu - m_p) <= 0.0101, (nb, mu)
