"""The library's network diagnostics (Assumption 3.4, Lemma 3.5; Sec. 6.1 and
6.2.1) against the oracle's (oracle/diagnostics.py, pinned by
test_oracle_diagnostics.py), a closed form, and the grid row of Table 6.3.

Host code: runs without a GPU. sigma and the box densities are sums in the
same order on both sides (1e-12); mu_box comes from Lanczos in the library and
from a dense or shift-invert eigensolver in the oracle (relative 1e-7); which
boxes cannot be joined within r0 (mu_box = inf) and which hold no edge
(mu_box = 0) must agree exactly."""
import numpy as np
import pytest

from paper_2207_07488_amd import workloads as W
import diagnostics as D  # oracle/diagnostics.py


@pytest.fixture(scope="module")
def S():
    from paper_2207_07488_amd import spnet
    try:
        spnet.lib()
    except (ImportError, OSError) as e:
        pytest.skip(f"libspnet not built: {e}")
    return spnet


def _compare(S, x, e, d, nb, r0=None):
    net = S.Network.from_arrays(x, e, d)
    sigma, mu, dens, mus = net.diagnostics(nb, r0)
    dd, so, _ = D.homogeneity(x, e, nb)
    mo, muo = D.connectivity(x, e, nb, r0)
    np.testing.assert_allclose(dens, dd, rtol=1e-12, atol=1e-12 * dd.max())
    if np.isfinite(so):
        assert sigma == pytest.approx(so, rel=1e-12)
    else:
        assert not np.isfinite(sigma)
    assert np.array_equal(np.isfinite(mus), np.isfinite(mo))
    assert np.array_equal(mus == 0, mo == 0)
    fin = np.isfinite(mo) & (mo > 0)
    np.testing.assert_allclose(mus[fin], mo[fin], rtol=1e-7)
    assert (mu == muo) if not np.isfinite(muo) else mu == pytest.approx(muo, rel=1e-7)
    return mus, mo


@pytest.mark.parametrize("n,nb", [(16, 4), (32, 8), (20, 3)])
def test_grid_matches_oracle(S, n, nb):
    x, e = W.grid_network(n)
    _compare(S, x, e, W.boundary_flags(x, 3, 3, 0.25 / n), nb)


@pytest.mark.parametrize("dim,nseg,length,nb,ce,r0", [
    (2, 400, 0.1, 8, 0.0, None),
    (2, 400, 0.1, 8, 0.0, 0.03),     # tight r0: some boxes cannot be joined
    (2, 2000, 0.05, 16, 0.0, None),  # empty boxes and boxes joined outside
    (3, 3000, 0.2, 4, 0.01, None),
])
def test_fiber_networks_match_oracle(S, dim, nseg, length, nb, ce, r0):
    """Sec. 6.1 fiber networks (seeded uniform centres and directions), sparse
    enough that boxes fall apart and must be joined through nodes within r0,
    or cannot be."""
    seg = W.fiber_segments(dim, nseg, length, 11)
    net = S.Network.from_segments(dim, seg, contact_eps=ce, merge_tol=W.merge_tol(length))
    x, e, d = net.arrays()
    mus, mo = _compare(S, x, e, d, nb, r0)
    if r0 is not None:
        assert not np.isfinite(mo).all()


def test_box_joined_outside(S):
    """The oracle's joining example: two edges in box (1, 1) of a 4 x 4 split
    meet only through a node 0.06 outside it; joined for r0 = 0.1 (mu_box as
    the oracle's lambda_2 of the joined subgraph), not for r0 = 0.03."""
    x = np.array([[0.30, 0.30], [0.45, 0.30], [0.30, 0.45], [0.45, 0.45], [0.52, 0.30], [0.52, 0.45],
                  [0.56, 0.375]])
    e = np.array([[0, 1], [2, 3], [1, 4], [3, 5], [4, 6], [5, 6]])
    d = np.zeros(len(x), dtype=np.uint8)
    net = S.Network.from_arrays(x, e, d)
    _, _, _, mus = net.diagnostics(4, 0.1)
    lam = D.lambda2(x, e, [0, 1, 2, 3, 4, 5])
    assert mus[5] == pytest.approx(1.0 / (0.25 * np.sqrt(lam)), rel=1e-9)
    assert mus[0] == 0.0  # no edge in box (0, 0)
    _, mu, _, mus = net.diagnostics(4, 0.03)
    assert not np.isfinite(mus[5]) and not np.isfinite(mu)


@pytest.mark.parametrize("m", [5, 17, 60, 400])
def test_lambda2_of_a_path(S, m):
    """A straight chain of m nodes with spacing h inside one box (nb = 1):
    lambda_2 = (2/h^2)(1 - cos(pi/(m-1))), mu = 1/sqrt(lambda_2)."""
    h = 0.5 / m
    x = np.stack([0.2 + h * np.arange(m), np.full(m, 0.5)], 1)
    e = np.stack([np.arange(m - 1), np.arange(1, m)], 1)
    net = S.Network.from_arrays(x, e, np.zeros(m, dtype=np.uint8))
    _, mu, _, _ = net.diagnostics(1)
    lam = 2 / h ** 2 * (1 - np.cos(np.pi / (m - 1)))
    assert mu == pytest.approx(1.0 / np.sqrt(lam), rel=1e-9)


def test_table_6_3_grid_row(S):
    """Table 6.3 (Sec. 6.2.1): sigma (1.0, 1.0, 1.1, 1.1) and mu (0.45, 0.47,
    0.48, 0.51) of the (2^9 + 1)^2 grid for H^-1 = 4, 8, 16, 32; sigma to its
    printed digit, mu to 0.01."""
    x, e = W.grid_network(512)
    net = S.Network.from_arrays(x, e, W.boundary_flags(x, 3, 3, 0.25 / 512))
    printed = {4: (1.0, 0.45), 8: (1.0, 0.47), 16: (1.1, 0.48), 32: (1.1, 0.51)}
    for nb, (s_p, m_p) in printed.items():
        sigma, mu, _, _ = net.diagnostics(nb)
        assert round(sigma, 1) == s_p, (nb, sigma)
        assert abs(mu - m_p) <= 0.0101, (nb, mu)


def test_errors(S):
    x, e = W.grid_network(4)
    net = S.Network.from_arrays(x, e, np.zeros(len(x), dtype=np.uint8))
    for nb, r0 in ((0, None), (2000, None), (4, float("nan")), (4, float("inf"))):
        with pytest.raises(S.SpnetError) as ei:
            net.diagnostics(nb, r0)
        assert ei.value.code == S.SN_EINVAL


@pytest.mark.slow
def test_table_6_1_uniform_instance(S):
    """The Sec. 6.1 uniform fiber network (fibers of length 0.05 until the
    clipped length reaches 1000, about 3.6e5 nodes), boxes B_R of side 2R for
    R^-1 = 16, joining paths within R0 = 1/64 (Table 6.1): the library's sigma,
    densities and mu_box match the oracle's on every box."""
    import os
    import sys
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
    import table_6_2 as T
    net = S.Network.from_segments(2, T.fiber_segments_sec61(), merge_tol=W.merge_tol(T.FIBER_LENGTH),
                                  dir_lo=3, dir_hi=3)
    x, e, d = net.arrays()
    _compare(S, x, e, d, 8, 1.0 / 64)
