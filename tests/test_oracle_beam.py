"""Pins of the oracle's beam model (Example 3.3: tensile eq. 3.4 plus bending
eq. 3.5, constants of Sec. 6.3), of its Dirichlet lifting and of the lumped
mass (eq. 2.1), against what mechanics and the paper fix:

* rigid motions carry no energy: translations, and rotations about the normal
  of a 2D network's plane (n = 2 and n = 3); in 3D every rotation, on
  networks whose neighbour pairs are all collinear (straight fibers). Checked
  through the lifting operator, (K g) on the free rows for g on every node;
* a straight cantilever (a chain clamped at one end by its first two nodes,
  loaded at the tip) converges to the Euler-Bernoulli tip deflection
  P L^3 / (3 EI') with EI' = gamma1 r_w^2 / 8 (the printed weights summed over
  ordered neighbour pairs), in 2D and along a skew line in 3D, in both
  transverse directions;
* K is symmetric and positive definite on V;
* lifting on the heat model equals the textbook graph Laplacian applied to g,
  and a linear field on a straight chain has no load at interior nodes;
* (M 1)(x) on the grid of Example 3.7 is 2/n inside, 1.5/n on edges."""
import numpy as np
import pytest

from paper_2207_07488_amd import workloads as W

G1 = 4.123e6   # A E for a steel wire of radius 2.5 mm (Sec. 6.3)
RW = 2.5e-3


def _chain(orc, n_seg, dim=2, direction=None, clamp=2):
    """Straight chain of n_seg edges of total length 1 from the origin along
    `direction`; the first `clamp` nodes are Dirichlet."""
    d = np.zeros(dim)
    d[0] = 1.0
    if direction is not None:
        d = np.asarray(direction, dtype=np.float64)
        d = d / np.linalg.norm(d)
    t = np.linspace(0.0, 1.0, n_seg + 1)
    x = 0.1 + t[:, None] * d[None, :]
    e = np.stack([np.arange(n_seg), np.arange(1, n_seg + 1)], 1).astype(np.int32)
    dirf = np.zeros(n_seg + 1, dtype=np.uint8)
    dirf[:clamp] = 1
    return orc.Network.from_arrays(x, e, dirf), x, d


def _fiber(orc, dim=2, n=150, l=0.25, seed=5, lo=1, hi=1):
    seg = W.fiber_segments(dim, n, l, seed=seed)
    return orc.Network.from_segments(dim, seg, contact_eps=0.02 if dim == 3 else 0.0, merge_tol=W.merge_tol(l),
                                     dir_lo=lo, dir_hi=hi)


@pytest.mark.parametrize("ncomp", [2, 3])
def test_rigid_motions_in_plane(orc, ncomp):
    net = _fiber(orc)
    x, _, _ = net.arrays()
    s = orc.System(net, orc.MODEL_BEAM, ncomp=ncomp, gamma1=G1, r_w=RW)
    K = s.dense()
    scale = np.abs(K).max()
    motions = [np.eye(ncomp)[0][None, :].repeat(len(x), 0), np.eye(ncomp)[1][None, :].repeat(len(x), 0)]
    rot = np.zeros((len(x), ncomp))
    rot[:, 0], rot[:, 1] = -x[:, 1], x[:, 0]
    motions.append(rot)
    if ncomp == 3:
        motions.append(np.eye(3)[2][None, :].repeat(len(x), 0))
    for g in motions:
        y = s.apply_full(g)
        assert np.abs(y).max() <= 1e-9 * scale * np.abs(g).max(), np.abs(y).max() / scale
    # a rotation about an in-plane axis does load the angled neighbour pairs (k = 1)
    tilt = np.zeros((len(x), 3))
    tilt[:, 2] = x[:, 1]
    if ncomp == 3:
        assert np.abs(s.apply_full(tilt)).max() > 1e-6 * scale


@pytest.mark.parametrize("direction", [(1.0, 0.0, 0.0), (0.3, -0.5, 0.8)])
def test_rigid_motions_straight_3d(orc, direction):
    """Straight chains in 3D: every rigid motion, rotations about any axis."""
    net, x, d = _chain(orc, 40, dim=3, direction=direction)
    s = orc.System(net, orc.MODEL_BEAM, ncomp=3, gamma1=G1, r_w=RW)
    scale = np.abs(s.dense()).max()
    for w in np.eye(3):
        g = np.cross(w[None, :], x - 0.37)
        assert np.abs(s.apply_full(g)).max() <= 1e-9 * scale * np.abs(g).max()
        g = np.repeat(w[None, :], len(x), 0)
        assert np.abs(s.apply_full(g)).max() <= 1e-9 * scale


@pytest.mark.parametrize("dim,direction", [(2, None), (3, (0.3, -0.5, 0.8))])
def test_cantilever_converges_to_euler_bernoulli(orc, dim, direction):
    """Tip deflection under a transverse tip load P: P L^3 / (3 EI') with
    EI' = gamma1 r_w^2 / 8, approached at first order in h (the clamp is two
    nodes); the load along the chain only stretches it: P L / gamma1."""
    P = 3.0
    errs = []
    for n_seg in (100, 200, 400):
        net, x, d = _chain(orc, n_seg, dim=dim, direction=direction)
        s = orc.System(net, orc.MODEL_BEAM, ncomp=dim if dim == 3 else 2, gamma1=G1, r_w=RW)
        K = s.dense()
        nc = s.ncomp
        normals = [np.array([-d[1], d[0]])] if dim == 2 else []
        if dim == 3:
            a = np.cross(d, [1.0, 0.0, 0.0])
            a /= np.linalg.norm(a)
            normals = [a, np.cross(d, a)]
        EI = G1 * RW ** 2 / 8
        L = 1.0
        for nv in normals:
            f = np.zeros(s.n)
            f[-nc:] = P * nv
            u = np.linalg.solve(K, f)
            tip = u[-nc:] @ nv
            errs.append((n_seg, abs(tip - P * L ** 3 / (3 * EI)) / (P * L ** 3 / (3 * EI))))
            # no coupling into the other directions
            assert abs(u[-nc:] @ d) <= 1e-9 * abs(tip)
        f = np.zeros(s.n)
        f[-nc:] = P * d
        u = np.linalg.solve(K, f)
        assert abs(u[-nc:] @ d - P * (L - L / n_seg) / G1) <= 1e-9 * P / G1
    e = {n: max(v for m, v in errs if m == n) for n, _ in errs}
    assert e[400] <= 0.01 and e[200] / e[400] > 1.8  # first order in h


@pytest.mark.parametrize("ncomp,dim", [(2, 2), (3, 2), (3, 3)])
def test_beam_operator_spd(orc, ncomp, dim):
    net = _fiber(orc, dim=dim, n=120 if dim == 2 else 300, l=0.25 if dim == 2 else 0.35,
                 lo=1 if dim == 2 else 4, hi=1 if dim == 2 else 4)
    s = orc.System(net, orc.MODEL_BEAM, ncomp=ncomp, gamma1=G1, r_w=RW)
    K = s.dense()
    assert np.array_equal(K, K.T) or np.abs(K - K.T).max() <= 1e-14 * np.abs(K).max()
    assert np.linalg.eigvalsh((K + K.T) / 2).min() > 0


def test_lifting_heat_is_graph_laplacian(orc):
    net = _fiber(orc)
    x, e, d = net.arrays()
    s = orc.System(net, 0)
    g = np.sin(3 * x[:, 0]) + x[:, 1] ** 2
    w = 1.0 / np.linalg.norm(x[e[:, 0]] - x[e[:, 1]], axis=1)
    lap = np.zeros(len(x))
    np.add.at(lap, e[:, 0], w * (g[e[:, 0]] - g[e[:, 1]]))
    np.add.at(lap, e[:, 1], w * (g[e[:, 1]] - g[e[:, 0]]))
    y = s.apply_full(g)
    ref = lap[s.free_nodes()]
    assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()
    # g supported on the free nodes only: the same as K restricted to V
    gf = np.zeros(len(x))
    gf[s.free_nodes()] = g[s.free_nodes()]
    assert np.abs(s.apply_full(gf) - s.apply_K(g[s.free_nodes()])).max() <= 1e-12 * np.abs(ref).max()


def test_lifting_linear_field_on_chain(orc):
    """g = (0.2 x_1, 0) on a straight chain with both ends fixed: uniform strain
    and no curvature, so the lifting load vanishes at every interior node."""
    net, x, d = _chain(orc, 30, dim=2, clamp=1)
    xx, e, dirf = net.arrays()
    dirf = dirf.copy()
    dirf[-1] = 1
    net = orc.Network.from_arrays(xx, e, dirf)
    s = orc.System(net, orc.MODEL_BEAM, ncomp=2, gamma1=G1, r_w=RW)
    g = np.zeros((len(xx), 2))
    g[:, 0] = 0.2 * xx[:, 0]
    assert np.abs(s.apply_full(g)).max() <= 1e-9 * G1


def test_mass_on_grid(orc):
    n = 8
    x, e = W.grid_network(n)
    net = orc.Network.from_arrays(x, e, W.boundary_flags(x, 1, 1, 0.25 / n))
    s = orc.System(net, 0)
    m = s.mass()
    fx = x[s.free_nodes()]
    inner = (fx[:, 1] > 0) & (fx[:, 1] < 1)
    assert np.allclose(m[inner], 2.0 / n, rtol=1e-14) and np.allclose(m[~inner], 1.5 / n, rtol=1e-14)
