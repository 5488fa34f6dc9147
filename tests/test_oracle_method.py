"""Pins of the oracle's operator, spaces, local/coarse solves and PCG.

Each check comes from the paper or from mathematics, not from re-typing the
oracle: the edge-sum form of eq. 3.3/3.4, the kernel of the Laplacian (Sec. 2.2),
reproduction of Q1 functions (Sec. 2.3), the literal half-open box membership of
the patches (Sec. 2.3), dense linear algebra, K-symmetry of BK (eq. 4.4), the
colouring bound on the spectrum of BK, monotone K-norm error (Sec. 4.2), the
Chebyshev bound (eq. 4.6) and a case with a closed-form answer.
"""
from fractions import Fraction

import numpy as np
import pytest

from paper_2207_07488_amd import workloads as W


def small_net(orc, n=300, l=0.2, seed=1, dim=2, lo=1, hi=1, eps=0.0):
    seg = W.fiber_segments(dim, n, l, seed=seed)
    return orc.Network.from_segments(dim, seg, contact_eps=eps, merge_tol=W.merge_tol(l), dir_lo=lo, dir_hi=hi)


def test_scalar_operator_edge_sum(orc):
    net = small_net(orc)
    x, e, d = net.arrays()
    s = orc.System(net, 0)
    K = s.dense()
    assert np.array_equal(K, K.T)  # bitwise symmetric
    fn = s.free_nodes()
    rng = np.random.default_rng(0)
    v = rng.standard_normal(s.n)
    vn = np.zeros(net.n_nodes)
    vn[fn] = v
    w = 1.0 / np.linalg.norm(x[e[:, 1]] - x[e[:, 0]], axis=1)
    q = np.sum(w * (vn[e[:, 0]] - vn[e[:, 1]]) ** 2)  # eq. 3.3 with gamma = 1
    assert abs(v @ K @ v - q) <= 1e-12 * q
    # kernel of the Laplacian: rows of nodes with no Dirichlet neighbour sum to zero
    nbr_dir = np.zeros(net.n_nodes, bool)
    nbr_dir[e[d[e[:, 1]] == 1, 0]] = True
    nbr_dir[e[d[e[:, 0]] == 1, 1]] = True
    rows = np.where(~nbr_dir[fn])[0]
    assert np.all(np.abs(K[rows].sum(1)) <= 1e-13 * np.diag(K)[rows])
    assert np.linalg.eigvalsh(K).min() > 0


def test_weighted_operator(orc):
    net = small_net(orc, seed=2)
    x, e, _ = net.arrays()
    g = 0.1 + 0.9 * W.uniform01(5, 0, net.n_edges)
    s = orc.System(net, 0, gamma=g)
    fn = s.free_nodes()
    v = np.sin(np.arange(s.n))
    vn = np.zeros(net.n_nodes)
    vn[fn] = v
    w = g / np.linalg.norm(x[e[:, 1]] - x[e[:, 0]], axis=1)
    q = np.sum(w * (vn[e[:, 0]] - vn[e[:, 1]]) ** 2)
    assert abs(v @ s.apply_K(v) - q) <= 1e-12 * q


def test_truss_operator(orc):
    net = small_net(orc, n=400, l=0.35, seed=3, dim=3, lo=4, hi=0, eps=0.03)
    x, e, d = net.arrays()
    s = orc.System(net, 1)
    assert s.n == 3 * s.n_free_nodes
    K = s.dense()
    assert np.array_equal(K, K.T)
    fn = s.free_nodes()
    rng = np.random.default_rng(1)
    v = rng.standard_normal(s.n)
    vn = np.zeros((net.n_nodes, 3))
    vn[fn] = v.reshape(-1, 3)
    dx = x[e[:, 1]] - x[e[:, 0]]
    ln = np.linalg.norm(dx, axis=1)
    t = dx / ln[:, None]
    dv = vn[e[:, 1]] - vn[e[:, 0]]
    q = np.sum((np.sum(dv * t, 1) ** 2 + 1e-6 * np.sum(dv * dv, 1)) / ln)  # eq. 3.4 + 1e-6 I term
    assert abs(v @ K @ v - q) <= 1e-11 * q
    # rigid translations are in the kernel away from the clamp
    nbr_dir = np.zeros(net.n_nodes, bool)
    nbr_dir[e[d[e[:, 1]] == 1, 0]] = True
    nbr_dir[e[d[e[:, 0]] == 1, 1]] = True
    free_rows = np.where(~nbr_dir[fn])[0]
    for c in range(3):
        tr = np.zeros(s.n)
        tr[c::3] = 1.0
        r = (K @ tr).reshape(-1, 3)[free_rows]
        assert np.abs(r).max() <= 1e-12 * np.abs(np.diag(K)).max()


def _in_support(xk, vk, nH):
    """Exact rational test |x_k nH - v_k| < 1: the hat factor of mesh node v_k
    is positive at x_k (Sec. 2.3)."""
    return abs(Fraction(xk) * nH - vk) < 1


def _grid(orc, n, lo, hi):
    """Example 3.7 grid network with Dirichlet faces lo/hi (bit k: axis k)."""
    x, e = W.grid_network(n)
    return orc.Network.from_arrays(x, e, W.boundary_flags(x, lo, hi, 0.25 / n))


_MEMBER_CASES = [("fiber", 2, 4, 0), ("fiber", 2, 3, 1), ("fiber", 3, 2, 0), ("grid", 2, 4, 0), ("grid", 2, 4, 1),
                 ("grid_x", 2, 4, 0), ("grid", 2, 3, 0)]


@pytest.mark.parametrize("kind,dim,nH,policy", _MEMBER_CASES)
def test_star_membership(orc, kind, dim, nH, policy):
    """Local space of mesh node y_v: the free nodes at which phi_v is positive
    (the support of phi_v, Sec. 4.1 and Sec. 5), by exact rational arithmetic.
    The grid networks put nodes on the faces of T_H (n = 8: every second grid
    line is a mesh line for nH = 4; nH = 3 puts none there), where a node lies
    only in the stars of the face's mesh nodes."""
    if kind == "fiber" and dim == 2:
        net, lo, hi = small_net(orc), 1, 1
    elif kind == "fiber":
        net, lo, hi = small_net(orc, n=300, l=0.35, dim=3, lo=4, hi=4, eps=0.03), 4, 4
    elif kind == "grid":
        net, lo, hi = _grid(orc, 8, 3, 3), 3, 3
    else:  # Dirichlet on x0 = 0, 1 only: free nodes on the faces x1 = 0 and x1 = 1
        net, lo, hi = _grid(orc, 8, 1, 1), 1, 1
    x, _, _ = net.arrays()
    s = orc.System(net, 0)
    p = orc.Precond(s, nH, policy, lo, hi, factor=False)
    sp, sd, sv = p.stars()
    fn = s.free_nodes()
    expect = {}
    for vid in range((nH + 1) ** dim):
        v = [(vid // (nH + 1) ** k) % (nH + 1) for k in range(dim)]
        on_gamma = any(((lo >> k) & 1 and v[k] == 0) or ((hi >> k) & 1 and v[k] == nH) for k in range(dim))
        if policy == 1 and on_gamma:
            continue
        mem = [i for i in range(len(fn)) if all(_in_support(x[fn[i], k], v[k], nH) for k in range(dim))]
        if mem:
            expect[vid] = mem
    assert list(sv) == sorted(expect)
    for j, vid in enumerate(sv):
        assert list(sd[sp[j]:sp[j + 1]]) == expect[vid]
    if policy == 0:
        # a node lies in 2 stars per axis where x_k nH is not an integer, else 1
        mult = [int(np.prod([1 if (Fraction(x[f, k]) * nH).denominator == 1 else 2 for k in range(dim)]))
                for f in fn]
        assert np.array_equal(np.bincount(sd, minlength=s.n), mult)
        if kind == "grid" and nH == 4:
            assert min(mult) == 1 and max(mult) == 4


def test_q1_reproduction_and_coarse_matrix(orc):
    # Gamma = {x0 = 0}: the bilinear g(x) = x0 (0.3 + 0.7 x1) vanishes on Gamma
    net = small_net(orc, lo=1, hi=0)
    x, _, _ = net.arrays()
    s = orc.System(net, 0)
    nH = 4
    p = orc.Precond(s, nH, 0, 1, 0)
    Pd = p.P_dense()
    assert Pd.min() >= 0.0 and Pd.max() <= 1.0
    cv = p.coarse_vertices()
    y = np.stack([(cv % (nH + 1)) / nH, (cv // (nH + 1)) / nH], 1)

    def g(z):
        return z[:, 0] * (0.3 + 0.7 * z[:, 1])

    fn = s.free_nodes()
    assert np.allclose(Pd @ g(y), g(x[fn]), rtol=0, atol=1e-14)
    # K0 = P^T K P, and c^T K0 c = v^T K v for v = P c
    K = s.dense()
    K0 = p.K0_dense()
    assert np.allclose(K0, Pd.T @ K @ Pd, rtol=0, atol=1e-11 * np.abs(K0).max())
    c = np.cos(np.arange(p.m0))
    vv = Pd @ c
    assert abs(c @ K0 @ c - vv @ K @ vv) <= 1e-11 * (vv @ K @ vv)


def test_coarse_dofs_with_boundary_values(orc):
    """Coarse dofs (Sec. 2.3): the mesh nodes off Gamma whose basis function is
    positive at some free node. Checked by brute force, and through a bilinear
    g that does not vanish on Gamma: the restricted coarse interpolant plus the
    Gamma nodes' terms, sum_v g(y_v) phi_v(x) with phi_v written out from the
    tensor hat, reproduces g at every free node."""
    net = small_net(orc, lo=1, hi=0)
    x, _, _ = net.arrays()
    s = orc.System(net, 0)
    nH = 4
    p = orc.Precond(s, nH, 0, 1, 0)
    fn = s.free_nodes()
    xf = x[fn]
    verts = [(a, b) for b in range(nH + 1) for a in range(nH + 1)]  # lexicographic, x fastest

    def phi(v, z):
        return np.maximum(0.0, 1 - np.abs(z[:, 0] * nH - v[0])) * np.maximum(0.0, 1 - np.abs(z[:, 1] * nH - v[1]))

    expect = [a + b * (nH + 1) for (a, b) in verts if a != 0 and (phi((a, b), xf) > 0).any()]
    cv = p.coarse_vertices()
    assert list(cv) == expect and p.m0 == len(expect)

    def g(z):
        return 0.5 + z[:, 0] + 0.3 * z[:, 1] + 0.2 * z[:, 0] * z[:, 1]

    y = np.stack([(cv % (nH + 1)) / nH, (cv // (nH + 1)) / nH], 1)
    gam = sum(g(np.array([[0.0, b / nH]]))[0] * phi((0, b), xf) for b in range(nH + 1))
    assert np.allclose(p.P_dense() @ g(y) + gam, g(xf), rtol=0, atol=1e-14)
    assert np.abs(gam).max() > 0.1  # the Gamma terms matter


def test_mesh_nodes_on_grid_nodes(orc):
    """Grid n = 6 with nH = 12: every grid node is a mesh node, whose support
    holds that node only; the mesh nodes between grid lines have no node in
    their support and are dropped. So P = I, K_0 = K, every local space is one
    node, and B = K^-1 + diag(K)^-1."""
    n, nH = 6, 12
    net = _grid(orc, n, 3, 3)
    s = orc.System(net, 0)
    p = orc.Precond(s, nH, 0, 3, 3)
    assert p.m0 == (n - 1) ** 2 and p.nstars == (n - 1) ** 2
    sp, sd, _ = p.stars()
    assert np.array_equal(np.diff(sp), np.ones(p.nstars, dtype=np.int64))
    assert np.array_equal(p.P_dense(), np.eye(s.n))
    K = s.dense()
    assert np.allclose(p.K0_dense(), K, rtol=0, atol=1e-12 * np.abs(K).max())
    r = np.cos(np.arange(s.n))
    ref = np.linalg.solve(K, r) + r / np.diag(K)
    assert np.allclose(p.apply_B(r), ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def _dense_B(p, n):
    return np.stack([p.apply_B(np.eye(n)[i]) for i in range(n)], 1)


def test_local_and_coarse_solves_are_exact(orc):
    net = small_net(orc)
    s = orc.System(net, 0)
    p = orc.Precond(s, 4)
    K = s.dense()
    sp, sd, _ = p.stars()
    rng = np.random.default_rng(3)
    for st in range(p.nstars):
        dofs = sd[sp[st]:sp[st + 1]]
        g = rng.standard_normal(len(dofs))
        z = p.star_solve(st, g)
        ref = np.linalg.solve(K[np.ix_(dofs, dofs)], g)
        assert np.linalg.norm(z - ref) <= 1e-10 * np.linalg.norm(ref)
    # B from the definition: P K0^{-1} P^T + sum_j R_j^T K_j^{-1} R_j
    Pd = p.P_dense()
    Bref = Pd @ np.linalg.solve(Pd.T @ K @ Pd, Pd.T)
    for st in range(p.nstars):
        dofs = sd[sp[st]:sp[st + 1]]
        Bref[np.ix_(dofs, dofs)] += np.linalg.inv(K[np.ix_(dofs, dofs)])
    B = _dense_B(p, s.n)
    assert np.abs(B - Bref).max() <= 1e-9 * np.abs(Bref).max()


def test_BK_symmetry_and_spectrum(orc):
    net = small_net(orc, n=300, l=0.2, seed=1)
    x, e, _ = net.arrays()
    s = orc.System(net, 0)
    nH = 4
    assert np.linalg.norm(x[e[:, 1]] - x[e[:, 0]], axis=1).max() < 1.0 / nH
    p = orc.Precond(s, nH)
    K = s.dense()
    B = _dense_B(p, s.n)
    assert np.abs(B - B.T).max() <= 1e-10 * np.abs(B).max()
    KBK = K @ B @ K  # (K P u, v) = (K u, P v), eq. 4.4
    assert np.abs(KBK - KBK.T).max() <= 1e-9 * np.abs(KBK).max()
    Lc = np.linalg.cholesky(K)
    lam = np.linalg.eigvalsh(Lc.T @ B @ Lc)
    # stars 3 apart in some index are K-orthogonal when edges are shorter than H:
    # 3^d colours of mutually orthogonal projections, plus the coarse projection
    assert lam.min() > 0 and lam.max() <= 3 ** 2 + 1 + 1e-9


def test_pcg_against_dense_direct_and_theory(orc):
    net = small_net(orc)
    s = orc.System(net, 0)
    p = orc.Precond(s, 4)
    K = s.dense()
    f = W.rhs(s.n, 1, seed=11)[:, 0]
    ustar = np.linalg.solve(K, f)
    u, it, info = p.pcg(f, rtol=1e-12, uref=ustar, history=True)
    assert np.linalg.norm(u - ustar) <= 1e-9 * np.linalg.norm(ustar)
    he = info["hist_e"]
    # CG minimises the K-norm error over nested Krylov spaces: non-increasing
    assert np.all(np.diff(he) <= 1e-12 * he[0])
    # Chebyshev bound, eq. 4.6, with kappa of BK
    B = _dense_B(p, s.n)
    Lc = np.linalg.cholesky(K)
    lam = np.linalg.eigvalsh(Lc.T @ B @ Lc)
    kap = lam.max() / lam.min()
    rate = (np.sqrt(kap) - 1) / (np.sqrt(kap) + 1)
    ells = np.arange(len(he))
    assert np.all(he <= 2 * rate ** ells * he[0] * (1 + 1e-8) + 1e-13 * he[0])
    # the true residual trails the recurrence only by rounding (residual gap)
    assert info["true_res"] <= 1e-10
    # fixed iteration count reproduces the stopped run
    u2, it2, _ = p.pcg(f, fixed_iters=it)
    assert it2 == it and np.array_equal(u2, u)


def test_single_element_one_step(orc):
    """nH = 1 on a grid with Dirichlet on all of the boundary: every free node
    lies strictly inside the one element, so each of the four local spaces is
    the whole space and the coarse space is empty (all mesh nodes on Gamma):
    BK = 4 I and PCG ends in one step with the exact solution."""
    net = _grid(orc, 8, 3, 3)
    s = orc.System(net, 0)
    p = orc.Precond(s, 1, 0, 3, 3)
    assert p.nstars == 4 and p.m0 == 0
    r = np.sin(np.arange(s.n))
    K = s.dense()
    assert np.allclose(p.apply_B(K @ r), 4 * r, rtol=0, atol=1e-12 * np.abs(r).max())
    f = W.rhs(s.n, 1, seed=2)[:, 0]
    u, it, info = p.pcg(f, rtol=1e-12)
    assert it == 1
    assert np.linalg.norm(K @ u - f) <= 1e-12 * np.linalg.norm(f)


@pytest.mark.slow
def test_iterations_bounded_under_refinement(orc):
    """Thm 4.3: at fixed H the rate does not depend on the number of nodes."""
    its = []
    for n in (300, 600, 1200, 2400):
        net = small_net(orc, n=n, l=0.2, seed=21)
        s = orc.System(net, 0)
        p = orc.Precond(s, 4)
        f = W.rhs(s.n, 1, seed=5)[:, 0]
        _, it, _ = p.pcg(f, rtol=1e-8)
        its.append(it)
    assert max(its) <= 1.5 * min(its), its
