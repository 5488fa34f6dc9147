"""Degenerate cases of the method on the GPU, each against the FP64 oracle:
a zero right-hand side (nothing to iterate), a mesh of one element with
Dirichlet data on the whole boundary (no coarse dof, every star the whole free
set: B = 4 K^-1 and PCG stops after one iteration), a network with a single free node (one star of one node, one
coarse dof), and sixteen columns on a system smaller than a wavefront.
"""
import numpy as np
import pytest

from paper_2207_07488_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2207_07488_amd import spnet
    spnet.lib()
    return spnet


def _fiber300(S, orc, nH, precision, faces=1):
    seg = W.fiber_segments(2, 300, 0.2, seed=1)
    tol = W.merge_tol(0.2)
    opre = orc.Precond(orc.System(orc.Network.from_segments(2, seg, merge_tol=tol, dir_lo=faces, dir_hi=faces), 0),
                       nH, 0, faces, faces)
    gpre = S.Precond(S.System(S.Network.from_segments(2, seg, merge_tol=tol, dir_lo=faces, dir_hi=faces)), nH, 0,
                     faces, faces, precision=precision)
    return opre, gpre


def _grid(S, orc, n, nH, precision):
    """Example 3.7 grid with (n+1)^2 nodes, Dirichlet on the whole boundary."""
    x, e = W.grid_network(n)
    d = W.boundary_flags(x, 3, 3, 1e-9)
    opre = orc.Precond(orc.System(orc.Network.from_arrays(x, e, d), 0), nH, 0, 3, 3)
    gpre = S.Precond(S.System(S.Network.from_arrays(x, e, d)), nH, 0, 3, 3, precision=precision)
    return opre, gpre


@pytest.mark.parametrize("prec", ["FP64", "FP32_STARS"])
def test_zero_right_hand_side(S, orc, prec):
    opre, gpre = _fiber300(S, orc, 4, getattr(S, prec))
    F = W.rhs(opre.sys.n, 3, seed=5)
    F[:, 1] = 0.0
    U, infos = gpre.solve(F, rtol=1e-8)
    assert np.all(U[:, 1] == 0.0)
    assert infos[1]["iters"] == 0 and infos[1]["converged"]
    for c in (0, 2):
        u1, i1 = gpre.solve(F[:, c], rtol=1e-8)
        assert np.array_equal(U[:, c], u1) and infos[c]["iters"] == i1[0]["iters"]
    u0, i0 = gpre.solve(np.zeros(opre.sys.n), rtol=1e-8)
    assert np.all(u0 == 0.0) and i0[0]["iters"] == 0


def test_one_element_mesh(S, orc):
    """H = 1 with Dirichlet on the whole boundary: all four mesh vertices lie on Gamma,
    so the coarse space is empty, and every basis function is positive at every free
    node, so every star holds every free node."""
    opre, gpre = _fiber300(S, orc, 1, S.FP64, faces=3)
    assert opre.m0 == 0 and gpre.m0 == 0
    assert opre.nstars == 4 and opre.star_total == 4 * opre.sys.n
    f = W.rhs(opre.sys.n, 1, seed=3)[:, 0]
    u_o, it_o, _ = opre.pcg(f, rtol=1e-8)
    u_g, info = gpre.solve(f, rtol=1e-8)
    assert it_o == 1 and info[0]["iters"] == 1
    assert np.max(np.abs(u_g - u_o)) <= 1e-10 * np.max(np.abs(u_o))
    r = W.rhs(opre.sys.n, 1, seed=4)[:, 0]
    z_g, z_o = gpre.apply_B(r), opre.apply_B(r)
    assert np.max(np.abs(z_g - z_o)) <= 1e-10 * np.max(np.abs(z_o))


@pytest.mark.parametrize("prec", ["FP64", "FP32_STARS"])
def test_single_free_node(S, orc, prec):
    """3 x 3 grid nodes, the centre free: K = 8 (four edges of weight 2), one star of
    one node, one coarse dof; u = f / 8."""
    opre, gpre = _grid(S, orc, 2, 2, getattr(S, prec))
    assert opre.sys.n == 1 and gpre.sys.n == 1
    f = np.array([0.7])
    u_o, it_o, _ = opre.pcg(f, rtol=1e-8)
    u_g, info = gpre.solve(f, rtol=1e-8)
    assert abs(u_g[0] - 0.7 / 8.0) <= 1e-15 and abs(u_o[0] - 0.7 / 8.0) <= 1e-15
    assert info[0]["iters"] == it_o
    U, infos = gpre.solve(np.full((1, 16), 0.7) * np.arange(1, 17), rtol=1e-8)
    assert np.allclose(U[0], 0.7 * np.arange(1, 17) / 8.0, rtol=1e-15, atol=0)


@pytest.mark.parametrize("prec", ["FP64", "FP32_STARS"])
def test_sixteen_columns_below_one_wavefront(S, orc, prec):
    """6 x 6 grid (25 free nodes), H = 1/3 (every mesh line runs through grid nodes):
    sixteen columns, each equal to its single solve bit for bit and to the oracle."""
    opre, gpre = _grid(S, orc, 6, 3, getattr(S, prec))
    assert opre.sys.n == 25
    F = W.rhs(opre.sys.n, 16, seed=21)
    U, infos = gpre.solve(F, rtol=1e-8)
    for c in range(16):
        u1, i1 = gpre.solve(F[:, c], rtol=1e-8)
        assert np.array_equal(U[:, c], u1) and infos[c]["iters"] == i1[0]["iters"]
        u_o, it_o, _ = opre.pcg(F[:, c], rtol=1e-8)
        if prec == "FP64":
            assert infos[c]["iters"] == it_o
            u_f, _ = gpre.solve(F[:, c], fixed_iters=it_o)
            assert np.max(np.abs(u_f - u_o)) <= 1e-10 * np.max(np.abs(u_o))
        assert infos[c]["converged"]
        res = np.linalg.norm(F[:, c] - opre.sys.apply_K(U[:, c])) / np.linalg.norm(F[:, c])
        assert res <= 1e-8
