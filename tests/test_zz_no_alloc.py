"""The entry point that allocates nothing (sn_apply_K_noalloc) against
sn_apply_K, through the C ABI: bit for bit, on two calls in a row, the second
with a smaller input (another, smaller network, fewer columns), so that the
second runs on a workspace the first has left full; and a request beyond the
workspace is refused with SN_EINVAL."""
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


def _precond(S, nseg, length, nH, seed):
    seg = W.fiber_segments(2, nseg, length, seed=seed)
    net = S.Network.from_segments(2, seg, merge_tol=W.merge_tol(length), dir_lo=1, dir_hi=1)
    return S.Precond(S.System(net), nH, S.STARS_ALL, 1, 1, precision=S.FP64)


def test_apply_K_noalloc_matches_apply_K(S):
    import torch
    big = _precond(S, 2000, 0.08, 8, 1)
    small = _precond(S, 300, 0.2, 4, 2)
    for pre, k, seed in ((big, 8, 3), (small, 1, 4)):
        x = W.rhs(pre.sys.n, k, seed=seed) - 0.5
        if k == 1:
            x = x[:, 0]
        ref = pre.apply_K(x)
        xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
        yd = torch.full_like(xd, float("nan"))
        pre.apply_K_noalloc(xd, yd)
        torch.cuda.synchronize()
        assert np.array_equal(yd.cpu().numpy(), ref), (pre.sys.n, k)


def test_apply_K_noalloc_refuses_beyond_workspace(S):
    import torch
    p = W.PRESETS["fiber2d_20k"]
    pre = _precond(S, p["n_segments"], p["length"], 32, p["seed"])
    # 2 * npad * 16 * 8 bytes of staging exceed the 64 MiB workspace
    x = torch.zeros((pre.sys.n, 16), dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(S.SpnetError) as ei:
        pre.apply_K_noalloc(x, y)
    assert ei.value.code == S.SN_EINVAL
