"""The device allocator hook (sn_set_allocator) on the GPU: with PyTorch's
caching allocator behind it the library computes the same bits as with
hipMalloc, hands back every block it took, and reports an allocator that
returns nothing as SN_ENOMEM.
"""
import gc

import numpy as np
import pytest

from paper_2207_07488_amd import workloads as W

pytestmark = pytest.mark.gpu

# 2000 segments of length 0.08 in the unit square, Dirichlet x = 0 and x = 1, H = 1/8
CASE = dict(dim=2, n_segments=2000, length=0.08, seed=1, dir_lo=1, dir_hi=1, nH=8)


@pytest.fixture(scope="module")
def S():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2207_07488_amd import spnet
    spnet.lib()
    yield spnet
    spnet.set_allocator(None, None)


def _precond(S, precision):
    c = CASE
    seg = W.fiber_segments(c["dim"], c["n_segments"], c["length"], seed=c["seed"])
    net = S.Network.from_segments(c["dim"], seg, merge_tol=W.merge_tol(c["length"]), dir_lo=c["dir_lo"],
                                  dir_hi=c["dir_hi"])
    return S.Precond(S.System(net), c["nH"], 0, c["dir_lo"], c["dir_hi"], precision=precision)


def _run(S, pre):
    F = W.rhs(pre.sys.n, 2, seed=11)
    u, infos = pre.solve(F, rtol=1e-8, use_graph=True)
    z = pre.apply_B(F[:, 0])
    return u, [i["iters"] for i in infos], z


def test_torch_allocator_same_bits_and_balanced(S):
    import torch
    ref = _precond(S, S.FP32_STARS)
    u0, it0, z0 = _run(S, ref)
    del ref
    gc.collect()

    live, count = {}, [0, 0]

    def alloc(nbytes, device):
        p = torch.cuda.caching_allocator_alloc(nbytes, device)
        live[p] = nbytes
        count[0] += 1
        return p

    def free(ptr, nbytes, device):
        assert live.pop(ptr) == nbytes
        count[1] += 1
        torch.cuda.caching_allocator_delete(ptr)

    S.set_allocator(alloc, free)
    try:
        pre = _precond(S, S.FP32_STARS)
        u1, it1, z1 = _run(S, pre)
        held = sum(live.values())
        assert count[0] > 0 and held > 0
        assert it1 == it0
        assert np.array_equal(u1, u0)
        assert np.array_equal(z1, z0)
        del pre
        gc.collect()
        torch.cuda.synchronize()
        assert not live, f"{len(live)} blocks ({sum(live.values())} bytes) not handed back"
        assert count[0] == count[1]
        print(f"allocator: {count[0]} blocks, {held / 2**20:.1f} MiB held by one preconditioner and engine")
    finally:
        S.set_allocator(None, None)


def test_allocator_out_of_memory_is_reported(S):
    S.set_allocator(lambda nbytes, device: 0, lambda ptr, nbytes, device: None)
    try:
        with pytest.raises(S.SpnetError) as ei:
            _precond(S, S.FP64)
        assert ei.value.code == S.SN_ENOMEM
    finally:
        S.set_allocator(None, None)
    pre = _precond(S, S.FP64)  # hipMalloc again
    u, it, _ = _run(S, pre)
    assert np.all(np.isfinite(u))


def test_use_torch_allocator_solves(S):
    import torch
    S.use_torch_allocator(True)
    try:
        before = torch.cuda.memory_allocated()
        pre = _precond(S, S.FP64)
        assert torch.cuda.memory_allocated() > before
        u, it, _ = _run(S, pre)
        assert all(i > 0 for i in it) and np.all(np.isfinite(u))
        del pre
        gc.collect()
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before
    finally:
        S.use_torch_allocator(False)
