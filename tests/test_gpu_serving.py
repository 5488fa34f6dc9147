"""Serving: continuous batching through the C ABI (sn_server_*).

Each request's result is the same, bit for bit, alone and in a mix of
requests on several networks that arrive while others iterate; it equals
sn_solve on the same right-hand sides, and it meets the tolerance against the
FP64 oracle.
"""
import numpy as np
import pytest

from paper_2207_07488_amd import workloads as W

pytestmark = pytest.mark.gpu

PROBLEMS = {
    # name: (dim, n_segments, length, contact_eps, dir_lo, dir_hi, nH)
    "p2d_small": (2, 300, 0.2, 0.0, 1, 1, 4),
    "p2d_2k": (2, 2000, 0.08, 0.0, 1, 1, 8),
    "p3d_6k": (3, 6000, 0.12, 0.012, 4, 4, 4),
}
# (problem, k, seed)
REQUESTS = [("p2d_2k", 3, 21), ("p3d_6k", 1, 22), ("p2d_small", 2, 23), ("p2d_2k", 1, 24),
            ("p3d_6k", 4, 25), ("p2d_2k", 4, 26), ("p2d_small", 1, 27), ("p3d_6k", 2, 28)]


@pytest.fixture(scope="module")
def S():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2207_07488_amd import spnet
    spnet.lib()
    return spnet


def _precond(S, name, factor=True):
    dim, nseg, l, eps, lo, hi, nH = PROBLEMS[name]
    seg = W.fiber_segments(dim, nseg, l, seed=5)
    net = S.Network.from_segments(dim, seg, contact_eps=eps, merge_tol=W.merge_tol(l), dir_lo=lo, dir_hi=hi)
    pre = S.Precond(S.System(net), nH, S.STARS_ALL, lo, hi)
    if factor:
        pre.factor(S.FP32_STARS)
    return pre


@pytest.fixture(scope="module")
def pres(S):
    return {name: _precond(S, name) for name in PROBLEMS}


def _rhs(pre, k, seed):
    return W.rhs(pre.sys.n, k, seed=seed)


def _drain(srv, tickets, max_steps=5000):
    out = {}
    for _ in range(max_steps):
        for t in list(tickets):
            r = srv.poll(t)
            if r is not None:
                out[t] = r
                tickets.remove(t)
        if not tickets:
            return out
        srv.step()
    raise AssertionError("server did not finish")


def _alone(S, pres):
    res = []
    for name, k, seed in REQUESTS:
        srv = S.Server(max_columns=8, iters_per_tick=4)
        t = srv.submit(pres[name], _rhs(pres[name], k, seed))
        res.append(_drain(srv, [t])[t])
        srv.close()
    return res


def test_same_alone_and_in_the_mix(S, pres):
    alone = _alone(S, pres)
    srv = S.Server(max_columns=8, iters_per_tick=4)
    tickets = []
    # requests arrive while earlier ones iterate
    for i, (name, k, seed) in enumerate(REQUESTS):
        tickets.append(srv.submit(pres[name], _rhs(pres[name], k, seed)))
        if i % 2 == 1:
            srv.step()
            srv.step()
    got = _drain(srv, list(tickets))
    for i, t in enumerate(tickets):
        u_mix, info_mix = got[t]
        u_alone, info_alone = alone[i]
        assert [x["iters"] for x in info_mix] == [x["iters"] for x in info_alone]
        assert np.array_equal(u_mix.reshape(u_alone.shape), u_alone), REQUESTS[i]
        assert all(x["converged"] for x in info_mix)


def test_server_thread_and_wait(S, pres):
    """The server's own host thread steps it (sn_server_run): requests submitted
    from this thread while it runs, some from a second Python thread, give the
    same results bit for bit as alone; sn_server_step is refused meanwhile;
    wait(0) returns once any result is ready; after the thread stops, wait()
    steps the server from the calling thread."""
    import threading
    alone = _alone(S, pres)
    srv = S.Server(max_columns=8, iters_per_tick=4)
    srv.run(True)
    srv.run(True)  # already running: no second thread
    with pytest.raises(S.SpnetError) as ei:
        srv.step()
    assert ei.value.code == S.SN_EBUSY
    tickets = [None] * len(REQUESTS)

    def submit(idx):
        for i in idx:
            name, k, seed = REQUESTS[i]
            tickets[i] = srv.submit(pres[name], _rhs(pres[name], k, seed))

    th = threading.Thread(target=submit, args=(range(1, len(REQUESTS), 2),))
    th.start()
    submit(range(0, len(REQUESTS), 2))
    th.join()
    assert srv.wait(0, timeout=120)
    got = {}
    for t in tickets:
        assert srv.wait(t, timeout=120)
        got[t] = srv.poll(t)
    for i, t in enumerate(tickets):
        u, info = got[t]
        u_alone, info_alone = alone[i]
        assert [x["iters"] for x in info] == [x["iters"] for x in info_alone]
        assert np.array_equal(u.reshape(u_alone.shape), u_alone), REQUESTS[i]
    srv.run(False)
    # without the thread, wait() steps the server itself
    name, k, seed = REQUESTS[0]
    t = srv.submit(pres[name], _rhs(pres[name], k, seed))
    assert srv.wait(t, timeout=120)
    u, info = srv.poll(t)
    assert np.array_equal(u.reshape(alone[0][0].shape), alone[0][0])
    assert not srv.wait(0, timeout=0.01)  # nothing pending
    srv.close()


def test_requests_admitted_together_into_one_engine(S, pres):
    """Several requests on one network submitted before a step start in the same
    engine at once; each converges as it does alone (regression: a later
    admission must not reset the start-up state of an earlier one)."""
    srv = S.Server(max_columns=8, iters_per_tick=4)
    pre = pres["p2d_2k"]
    F = [_rhs(pre, k, 60 + k) for k in (3, 2, 1, 2)]
    tickets = [srv.submit(pre, f) for f in F]
    got = _drain(srv, list(tickets))
    for f, t in zip(F, tickets):
        u, infos = got[t]
        u1, i1 = pre.solve(f, rtol=1e-8)
        assert all(x["converged"] and x["iters"] < 200 for x in infos)
        assert [x["iters"] for x in infos] == [x["iters"] for x in i1]
        assert np.array_equal(u.reshape(u1.shape), u1)


def test_server_matches_sn_solve_and_oracle(S, pres, orc):
    srv = S.Server(max_columns=8, iters_per_tick=4)
    name, k, seed = "p2d_2k", 3, 31
    pre = pres[name]
    F = _rhs(pre, k, seed)
    t = srv.submit(pre, F)
    u, infos = _drain(srv, [t])[t]
    u_s, infos_s = pre.solve(F, rtol=1e-8)
    assert np.array_equal(u, u_s)
    assert [x["iters"] for x in infos] == [x["iters"] for x in infos_s]
    dim, nseg, l, eps, lo, hi, nH = PROBLEMS[name]
    seg = W.fiber_segments(dim, nseg, l, seed=5)
    on = orc.Network.from_segments(dim, seg, contact_eps=eps, merge_tol=W.merge_tol(l), dir_lo=lo, dir_hi=hi)
    opre = orc.Precond(orc.System(on), nH, 0, lo, hi)
    for c in range(k):
        u_o, _, _ = opre.pcg(F[:, c], rtol=1e-8)
        assert infos[c]["res_true"] <= 1.0001e-8
        assert np.linalg.norm(u[:, c] - u_o) / np.linalg.norm(u_o) <= 1e-5


def test_server_factors_and_evicts_within_budget(S):
    """A budget that holds one of two similar networks at a time: the server
    factors both (host worker threads), serves one network after the other
    and evicts the idle engine and the factors it uploaded; results equal
    those of preconditioners factored by the caller."""
    def pre_seed(seed, factor):
        dim, nseg, l, eps, lo, hi, nH = PROBLEMS["p2d_2k"]
        seg = W.fiber_segments(dim, nseg, l, seed=seed)
        net = S.Network.from_segments(dim, seg, merge_tol=W.merge_tol(l), dir_lo=lo, dir_hi=hi)
        pre = S.Precond(S.System(net), nH, S.STARS_ALL, lo, hi)
        if factor:
            pre.factor(S.FP32_STARS)
        return pre

    kc = 4
    ref, sizes = {}, []
    for seed in (5, 6):
        pre = pre_seed(seed, True)
        srv = S.Server(max_columns=kc)
        t = srv.submit(pre, _rhs(pre, 2, 41))
        ref[seed] = _drain(srv, [t])[t][0]
        srv.close()
        npad = (pre.sys.n + 255) // 256 * 256
        sizes.append(pre.factor_info()["device_bytes"] + (6 * npad * kc + pre.star_total * kc) * 8)
    budget = int(1.5 * max(sizes))
    a, b = pre_seed(5, False), pre_seed(6, False)
    srv = S.Server(hbm_budget=budget, max_columns=kc)
    ta = srv.submit(a, _rhs(a, 2, 41))
    tb = srv.submit(b, _rhs(b, 2, 41))
    out, peak, engines = {}, 0, 0
    for _ in range(20000):
        srv.step()
        used, neng = srv.usage()
        peak, engines = max(peak, used), max(engines, neng)
        for t in (ta, tb):
            if t not in out:
                r = srv.poll(t)
                if r is not None:
                    out[t] = r
        if len(out) == 2:
            break
    assert len(out) == 2
    assert peak <= budget and engines == 1
    assert np.array_equal(out[ta][0], ref[5])
    assert np.array_equal(out[tb][0], ref[6])


def test_server_rejects_oversized_requests(S, pres):
    srv = S.Server(hbm_budget=1 << 20, max_columns=2)
    with pytest.raises(S.SpnetError) as ei:
        srv.submit(pres["p2d_2k"], _rhs(pres["p2d_2k"], 1, 1))
    assert ei.value.code == S.SN_EBUSY
    with pytest.raises(S.SpnetError) as ei:
        srv.submit(pres["p2d_2k"], _rhs(pres["p2d_2k"], 3, 1))
    assert ei.value.code == S.SN_EINVAL


def test_failed_factorisation_fails_only_that_request(S, pres):
    """A request whose preconditioner cannot be factored (one element, nH = 1,
    on a 301 x 301 grid: its local spaces hold 90,000 dofs, beyond the 65,535
    positions a star may have; the check runs in the host factor worker before
    any device work) fails alone: the requests queued beside it still
    complete, and the failed one reports its error once."""
    x, e = W.grid_network(300)
    net = S.Network.from_arrays(x, e, W.boundary_flags(x, 1, 1, 1e-4))
    bad = S.Precond(S.System(net), 1, S.STARS_ALL, 1, 1)
    srv = S.Server(max_columns=4)
    tb = srv.submit(bad, _rhs(bad, 1, 1))
    good = [srv.submit(pres["p2d_2k"], _rhs(pres["p2d_2k"], 2, 51)),
            srv.submit(pres["p3d_6k"], _rhs(pres["p3d_6k"], 1, 52))]
    failed = None
    done = {}
    for _ in range(5000):
        srv.step()
        if failed is None:
            try:
                srv.poll(tb)
            except S.SpnetError as e:
                failed = e
        for t in good:
            if t not in done:
                r = srv.poll(t)
                if r is not None:
                    done[t] = r
        if failed is not None and len(done) == 2:
            break
    assert failed is not None and failed.code == S.SN_EINVAL and "65536 or more dofs" in str(failed)
    assert len(done) == 2
    for u, infos in done.values():
        assert all(x["converged"] and x["res_true"] <= 1.0001e-8 for x in infos)
