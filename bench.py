#!/usr/bin/env python3
"""PCG solves/s at rtol 1e-8 on one MI355X: two-level additive Schwarz PCG on a
2D fiber network (20,000 segments of length 0.05 in the unit square, Dirichlet
at x = 0 and x = 1, f uniform[0,1], H = 1/64 by default; H = 1/16 and 1/32 in
the mesh-size sweep), mixed form (FP32 local solves, FP64 coarse operator and
CG) against the plain FP64 form, with p50/p99 latency per solve.

A step is one full PCG solve (u0 = 0 to ||r|| <= 1e-8 ||f||) of one right-hand
side already resident in HBM, iterations replayed from captured HIP graphs.
Beside the headline: the mesh-size sweep, batched right-hand sides, the small
2D network with 1,024 right-hand sides, the 3D fiber network (100,000
segments), the 3D truss network with 16 right-hand sides, the heat experiment
of Sec. 6.2 on the Example 3.7 grid, the in-plane structural problem of Sec.
6.3.1 (beam model, lifted Dirichlet data), the network diagnostics of
Assumption 3.4 (host), the serving mix, and the FP64
oracle timed on the host (one core and all cores). Prints one JSON
line; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_F64_TFLOPS = 78.6
KERNEL_SOURCES = ("paper_2207_07488_amd/csrc/star_band.hpp", "paper_2207_07488_amd/csrc/star_sn.hpp",
                  "paper_2207_07488_amd/csrc/star_inst.hip", "paper_2207_07488_amd/csrc/device_common.hpp")


def kernel_source_hash():
    """Hash of the local-solve kernel sources: counter data taken on other sources is stale."""
    import hashlib
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q
    lo, hi = int(k), min(int(k) + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def timed_solves(pre, f, steps, warmup, rtol, profile=False, use_graph=False):
    import torch
    from paper_2207_07488_amd import spnet as S
    for _ in range(warmup):
        pre.solve(f, rtol=rtol, use_graph=use_graph)
    torch.cuda.synchronize()
    if profile:
        S._check(S.lib().sn_precond_profile(pre.h, 1))
    lat, iters = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u = None
    for _ in range(steps):
        a = time.perf_counter()
        u, info = pre.solve(f, rtol=rtol, use_graph=use_graph)
        lat.append((time.perf_counter() - a) * 1e3)
        iters.append(info[0]["iters"])
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    stats = None
    if profile:
        st = S.KernelStats()
        S._check(S.lib().sn_precond_kernel_stats(pre.h, S.C.byref(st)))
        S._check(S.lib().sn_precond_profile(pre.h, 0))
        stats = st.asdict()
    return dict(total_s=total, lat_ms=lat, iters=iters, u=u, info=info, stats=stats)


def copy_probe(mib):
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8, "launches": 5}), flush=True)


def serving_leg(n_requests, rate, pool_size=8, seed=5, load=0.7):
    """Poisson arrivals of solve requests (1-8 right-hand sides, uniform[0,1]
    loads) on a pool of 2D and 3D fiber networks of 2k-500k nodes, served by
    one continuous-batching server (FP32 stars). The pool's factors are made
    resident by one untimed request per network first. First the saturation
    throughput: every request submitted at once. Then arrivals at `load` times
    that request rate (or at `rate` if given); latency runs from the scheduled
    arrival to the poll that returns the result. The server's own host thread
    steps it; the benchmark thread only submits and collects."""
    import numpy as np
    from paper_2207_07488_amd import spnet as S
    from paper_2207_07488_amd import workloads as W
    pool = W.serving_pool(pool_size, seed)
    pres = []
    for p in pool:
        seg = W.fiber_segments(p["dim"], p["n_segments"], p["length"], p["seed"])
        net = S.Network.from_segments(p["dim"], seg, contact_eps=p.get("contact_eps", 0.0),
                                      merge_tol=W.merge_tol(p["length"]), dir_lo=p["dir_lo"], dir_hi=p["dir_hi"],
                                      band=W.BAND)
        pres.append(S.Precond(S.System(net), p["nH"], S.STARS_ALL, p["dir_lo"], p["dir_hi"]))
    srv = S.Server(max_columns=8, iters_per_tick=4, precision=S.FP32_STARS)
    srv.run(True)
    # resident factors, engines and captured graphs (untimed)
    warm = [srv.submit(pre, W.rhs(pre.sys.n, 1, seed=1)) for pre in pres]
    for t in warm:
        if not srv.wait(t, timeout=600):
            raise RuntimeError("serving warm-up did not finish")
        srv.poll(t)
    pick = W.uniform01(seed + 2, 0, 2 * n_requests)
    reqs = []
    for i in range(n_requests):
        j = min(int(pick[2 * i] * len(pres)), len(pres) - 1)
        k = 1 + min(int(pick[2 * i + 1] * 8), 7)
        reqs.append((j, k, W.rhs(pres[j].sys.n, k, seed=100 + i)))

    def run(arrivals):
        # the server's own host thread steps it; this thread submits at the
        # arrival times and collects results as they become ready
        pending, lat, iters, worst = {}, [], [], 0.0
        nxt, solved = 0, 0
        t0 = time.perf_counter()
        while nxt < n_requests or pending:
            now = time.perf_counter() - t0
            while nxt < n_requests and arrivals[nxt] <= now:
                j, k, F = reqs[nxt]
                pending[srv.submit(pres[j], F)] = (nxt, k)
                nxt += 1
            wait_s = arrivals[nxt] - (time.perf_counter() - t0) if nxt < n_requests else 60.0
            if pending:
                if not srv.wait(0, timeout=max(0.0, wait_s)):
                    continue
            else:
                time.sleep(max(0.0, wait_s))
                continue
            for t in list(pending):
                r = srv.poll(t)
                if r is None:
                    continue
                i, k = pending.pop(t)
                lat.append((time.perf_counter() - t0 - arrivals[i]) * 1e3)
                iters.extend(x["iters"] for x in r[1])
                worst = max(worst, max(x["res_true"] for x in r[1]))
                solved += k
        return time.perf_counter() - t0, lat, iters, worst, solved

    run(np.zeros(n_requests))  # untimed pass: every engine's graphs and tick shapes exist afterwards
    sat_s, sat_lat, _, _, solved = run(np.zeros(n_requests))
    sat_req_rate = n_requests / sat_s
    arr_rate = rate if rate and rate > 0 else load * sat_req_rate
    arrivals = W.poisson_arrivals(n_requests, arr_rate, seed + 1)
    makespan, lat, iters, worst, solved = run(arrivals)
    used, neng = srv.usage()
    srv.run(False)
    srv.close()
    return {"requests": n_requests, "rhs_solved": solved,
            "saturation": {"solves_per_s": round(solved / sat_s, 2), "requests_per_s": round(sat_req_rate, 2),
                           "latency_ms": {"p50": round(percentile(sat_lat, 0.5), 3),
                                          "p99": round(percentile(sat_lat, 0.99), 3)}},
            "poisson": {"arrival_rate_per_s": round(arr_rate, 2), "load": None if rate else load,
                        "solves_per_s": round(solved / makespan, 2), "makespan_s": round(makespan, 3),
                        "latency_ms": {"p50": round(percentile(lat, 0.5), 3), "p99": round(percentile(lat, 0.99), 3)}},
            "median_iterations": int(np.median(iters)), "max_res_true": worst,
            "networks": [{"dim": p["dim"], "dofs": pre.sys.n, "nH": p["nH"], "stars": pre.nstars} for p, pre in
                         zip(pool, pres)],
            "engines": neng, "device_bytes": used, "engine_width": 8, "iters_per_tick": 4}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def build_problem(S, W, preset, nH, precision, model=None):
    p = dict(preset)
    seg = W.fiber_segments(p["dim"], p["n_segments"], p["length"], p["seed"])
    net = S.Network.from_segments(p["dim"], seg, contact_eps=p.get("contact_eps", 0.0),
                                  merge_tol=W.merge_tol(p["length"]), dir_lo=p["dir_lo"], dir_hi=p["dir_hi"],
                                  band=W.BAND)
    sysm = S.System(net, p.get("model", 0) if model is None else model)
    pre = S.Precond(sysm, nH, S.STARS_ALL, p["dir_lo"], p["dir_hi"], precision=precision)
    return seg, net, sysm, pre


def rate(n, seconds):
    return round(n / seconds, 3)


def c1_leg(S, W, torch, steps):
    """The small 2D network (300 segments, H = 1/4) with 1,024 right-hand sides:
    plain FP64 one column at a time, and the mixed form 16 columns per batch."""
    p = W.PRESETS["fiber2d_300"]
    _, net, sysm, plain = build_problem(S, W, p, p["nH"], S.FP64)
    mixed = S.Precond(sysm, p["nH"], S.STARS_ALL, p["dir_lo"], p["dir_hi"], precision=S.FP32_STARS)
    F = torch.from_numpy(W.rhs(sysm.n, 1024, seed=0)).cuda()
    cols = [F[:, j].contiguous() for j in range(1024)]
    batches = [F[:, 16 * b:16 * b + 16].contiguous() for b in range(64)]
    out = {"workload": "fiber2d_300_H4", "dofs": sysm.n, "rhs": 1024}
    for name, pre, blocks, k in (("plain_one_at_a_time", plain, cols, 1), ("mixed_16_per_batch", mixed, batches, 16)):
        pre.solve(blocks[0], rtol=1e-8, use_graph=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        iters = []
        for b in blocks:
            _, info = pre.solve(b, rtol=1e-8, use_graph=True)
            iters.append(max(i["iters"] for i in info))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[name] = {"solves_per_s": rate(len(blocks) * k, dt), "s": round(dt, 3), "max_iterations": max(iters)}
    return out


def c3_leg(S, W, torch, steps):
    """3D fiber network: 100,000 segments of length 0.05, contact 0.005,
    Dirichlet z = 0, 1, H = 1/16; mixed and plain, one right-hand side."""
    p = W.PRESETS["fiber3d_100k"]
    t0 = time.perf_counter()
    _, net, sysm, mixed = build_problem(S, W, p, 16, S.FP32_STARS)
    setup = time.perf_counter() - t0
    plain = S.Precond(sysm, 16, S.STARS_ALL, p["dir_lo"], p["dir_hi"], precision=S.FP64)
    f = torch.from_numpy(W.rhs(sysm.n, 1, seed=7)[:, 0]).cuda()
    out = {"workload": "fiber3d_100k_H16", "nodes": net.n_nodes, "dofs": sysm.n, "stars": mixed.nstars,
           "m0": mixed.m0, "setup_s": round(setup, 2)}
    for name, pre in (("mixed", mixed), ("plain", plain)):
        r = timed_solves(pre, f, max(3, steps // 5), 1, 1e-8, use_graph=True)
        out[name] = {"solves_per_s": rate(len(r["iters"]), r["total_s"]), "iterations": int(r["iters"][-1]),
                     "res_true": r["info"][0]["res_true"], "engine": pre.engine_info(1)}
    fi = mixed.factor_info()
    out["factor"] = {k: fi[k] for k in ("star_factor_nnz", "star_rcm_nnz", "max_star_dofs", "max_levels",
                                        "star_precision", "factor_seconds")}
    return out


def c4_leg(S, W, torch, steps):
    """3D truss network (3 dofs per node): 30,000 segments of length 0.1 of the
    3D geometry, clamp z = 0, f uniform[-1, 1], H = 1/16, 16 right-hand sides per
    solve (FP32 local solves requested; the library keeps FP64 where FP32
    cannot resolve them). The coarse product is a 16-column GEMM on the FP64
    matrix cores: its MFMA utilisation is reported."""
    p = W.PRESETS["truss3d_30k"]
    t0 = time.perf_counter()
    _, net, sysm, pre = build_problem(S, W, p, 16, S.FP32_STARS)
    setup = time.perf_counter() - t0
    F = torch.from_numpy(W.rhs(sysm.n, 16, seed=9, lo=-1.0, hi=1.0)).cuda()
    fi = pre.factor_info()
    out = {"workload": "truss3d_30k_H16_16rhs", "nodes": net.n_nodes, "dofs": sysm.n, "stars": pre.nstars,
           "m0": pre.m0, "setup_s": round(setup, 2), "star_precision": fi["star_precision"],
           "max_pivot_ratio": fi["max_pivot_ratio"]}
    U, info = pre.solve(F, rtol=1e-8, use_graph=True, raise_on_noconv=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    U, info = pre.solve(F, rtol=1e-8, use_graph=True, raise_on_noconv=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out["solves_per_s"] = rate(16, dt)
    out["s_per_batch"] = round(dt, 3)
    out["iterations"] = [int(i["iters"]) for i in info]
    out["converged"] = all(i["converged"] for i in info)
    out["max_res_true"] = max(i["res_true"] for i in info)
    # the coarse product alone: timed kernel launches over a few iterations
    S._check(S.lib().sn_precond_profile(pre.h, 1))
    pre.solve(F, fixed_iters=4, use_graph=False)
    st = S.KernelStats()
    S._check(S.lib().sn_precond_kernel_stats(pre.h, S.C.byref(st)))
    S._check(S.lib().sn_precond_profile(pre.h, 0))
    st = st.asdict()
    if st["coarse_launches"]:
        us = st["coarse_ms"] / st["coarse_launches"] * 1e3
        tflops = 16 * st["coarse_flops"] / (us * 1e-6) / 1e12
        out["coarse_product"] = {"us": round(us, 2), "columns": 16, "flops": 16 * st["coarse_flops"],
                                 "tflops": round(tflops, 2), "peak_tflops": PEAK_F64_TFLOPS,
                                 "mfma_utilisation": round(tflops / PEAK_F64_TFLOPS, 4),
                                 "bytes": 8 * pre.m0 * pre.m0, "hbm_frac": round(8 * pre.m0 * pre.m0 / (us * 1e-6) / 1e9 / PEAK_HBM_GBS, 4)}
    if st["sweep_launches"]:
        out["local_solves_us"] = round(st["sweep_ms"] / st["sweep_launches"] * 1e3, 2)
    return out


def f1_leg(S, W, torch):
    """The heat experiment of Sec. 6.2 on the GPU: the Example 3.7 grid with
    (2^9 + 1)^2 nodes, f = M1, Dirichlet on all of the boundary, FP64 and mixed
    solves at H^-1 = 4 .. 32 (the rates of Table 6.2 are pinned by the tests;
    here: iterations and throughput)."""
    x, e = W.grid_network(512)
    net = S.Network.from_arrays(x, e, W.boundary_flags(x, 3, 3, 0.25 / 512))
    sysm = S.System(net)
    f = torch.from_numpy(sysm.mass()).cuda()
    out = {"workload": "grid_513x513_f_M1", "dofs": sysm.n}
    for nH in (4, 8, 16, 32):
        row = {}
        for name, prec in (("plain", S.FP64), ("mixed", S.FP32_STARS)):
            pre = S.Precond(sysm, nH, S.STARS_ALL, 3, 3, precision=prec)
            pre.solve(f, rtol=1e-8, use_graph=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                _, info = pre.solve(f, rtol=1e-8, use_graph=True)
            torch.cuda.synchronize()
            row[name] = {"solves_per_s": rate(3, time.perf_counter() - t0), "iterations": int(info[0]["iters"]),
                         "res_true": info[0]["res_true"], "max_star_dofs": pre.factor_info()["max_star_dofs"]}
            del pre
        out[f"H=1/{nH}"] = row
    return out


def f2_leg(S, W, torch):
    """The in-plane tensile problem of Sec. 6.3.1 on the 20,000-segment 2D
    network: beam model (eq. 3.4 + eq. 3.5, steel wire of radius 2.5 mm,
    gamma1 = A E), Gamma = {x_1 = 0 or 1}, u-hat = u + g with g = (0.2 x_1, 0),
    f = -(K g); FP64 and mixed solves at H = 1/16 and 1/32. rate_est is the
    mean residual reduction per iteration, (1e-8)^(1/iterations)."""
    import numpy as np
    p = W.PRESETS["fiber2d_20k"]
    seg = W.fiber_segments(2, p["n_segments"], p["length"], p["seed"])
    net = S.Network.from_segments(2, seg, merge_tol=W.merge_tol(p["length"]), dir_lo=1, dir_hi=1, band=W.BAND)
    g1 = 3.141592653589793 * 2.5e-3 ** 2 * 210e9
    sysm = S.System(net, S.MODEL_BEAM, ncomp=2, gamma1=g1, r_w=2.5e-3)
    x, _, _ = net.arrays()
    g = np.zeros((net.n_nodes, 2))
    g[:, 0] = 0.2 * x[:, 0]
    f = torch.from_numpy(-sysm.apply_full(g)).cuda()
    out = {"workload": "struct2d_20k_tensile", "dofs": sysm.n, "nnz": sysm.nnz}
    for nH in (16, 32):
        row = {}
        for name, prec in (("plain", S.FP64), ("mixed", S.FP32_STARS)):
            pre = S.Precond(sysm, nH, S.STARS_ALL, 1, 1, precision=prec)
            pre.solve(f, rtol=1e-8, max_iter=2000, use_graph=True, raise_on_noconv=False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info = pre.solve(f, rtol=1e-8, max_iter=2000, use_graph=True, raise_on_noconv=False)
            torch.cuda.synchronize()
            it = int(info[0]["iters"])
            row[name] = {"solves_per_s": rate(1, time.perf_counter() - t0), "iterations": it,
                         "converged": bool(info[0]["converged"]), "res_true": info[0]["res_true"],
                         "rate_est": round(1e-8 ** (1.0 / max(it, 1)), 3),
                         "star_precision": pre.factor_info()["star_precision"]}
            del pre
        out[f"H=1/{nH}"] = row
    return out


def f4_leg(S, W, torch):
    """Network diagnostics of Assumption 3.4 (host code of the library): sigma
    and mu of the Example 3.7 grid with (2^9 + 1)^2 nodes over boxes of side H
    (Table 6.3) and of the 20,000-segment 2D network over boxes of side 2R with
    joining paths within 1/64 (the measure of Table 6.1), with their times."""
    x, e = W.grid_network(512)
    grid = S.Network.from_arrays(x, e, W.boundary_flags(x, 3, 3, 0.25 / 512))
    p = W.PRESETS["fiber2d_20k"]
    seg = W.fiber_segments(2, p["n_segments"], p["length"], p["seed"])
    fib = S.Network.from_segments(2, seg, merge_tol=W.merge_tol(p["length"]), dir_lo=3, dir_hi=3, band=W.BAND)
    out = {"grid_513x513": {}, "fiber2d_20k": {}}
    for name, net, sizes, r0 in (("grid_513x513", grid, (4, 8, 16, 32), None),
                                 ("fiber2d_20k", fib, (2, 4, 8, 16, 32), 1.0 / 64)):
        for nb in sizes:
            t0 = time.perf_counter()
            sigma, mu, _, _ = net.diagnostics(nb, r0)
            key = f"H=1/{nb}" if r0 is None else f"R=1/{2 * nb}"
            out[name][key] = {"sigma": round(sigma, 3), "mu": round(mu, 3),
                              "seconds": round(time.perf_counter() - t0, 3)}
    return out


def cpu_oracle_leg(O, W, seg, tol, preset, nH, f_host, rtol, threads):
    """The FP64 oracle on the host: one solve on one core, and independent
    solves (other right-hand sides of the same network) on `threads` cores at
    once (the oracle is single threaded; the C calls release the GIL)."""
    from concurrent.futures import ThreadPoolExecutor
    import numpy as np
    onet = O.Network.from_segments(2, seg, merge_tol=tol, dir_lo=preset["dir_lo"], dir_hi=preset["dir_hi"],
                                   band=W.BAND)
    opre = O.Precond(O.System(onet), nH, 0, preset["dir_lo"], preset["dir_hi"])
    md_nnz = opre.star_md_nnz()
    t0 = time.perf_counter()
    u_o, it_o, _ = opre.pcg(f_host, rtol=rtol)
    t1 = time.perf_counter() - t0
    F = W.rhs(len(f_host), threads, seed=101)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(lambda j: opre.pcg(np.ascontiguousarray(F[:, j]), rtol=rtol), range(threads)))
    tn = time.perf_counter() - t0
    return u_o, it_o, t1, threads / tn, tn, md_nnz


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--nH", type=int, default=64)
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-h-sweep", action="store_true")
    ap.add_argument("--no-configs", action="store_true", help="skip the other workloads (c1, c3, c4)")
    ap.add_argument("--serving-requests", type=int, default=64)
    ap.add_argument("--serving-rate", type=float, default=0.0,
                    help="Poisson arrival rate (requests/s); 0: 70%% of the measured saturation rate")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic_local_solves_fiber2d_20k_H64.json"),
                    help="HBM traffic per local-solve launch from rocprofv3 counters (JSON), if present")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (5 times) and exit: the reference "
                         "kernel that scales the FETCH_SIZE / WRITE_SIZE counters to bytes")
    ap.add_argument("--only-apply-b", type=int, default=0, metavar="N",
                    help="only set up the headline workload (mixed form) and apply B N times, then exit (the "
                         "short program the hardware-counter passes profile)")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2207_07488_amd import spnet as S
    from paper_2207_07488_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    preset = dict(W.PRESETS["fiber2d_20k"])
    t_setup = time.perf_counter()
    seg, net, sysm, mixed = build_problem(S, W, preset, args.nH, S.FP32_STARS)
    t_setup = time.perf_counter() - t_setup
    tol = W.merge_tol(preset["length"])
    f_host = W.rhs(sysm.n, 1, seed=7)[:, 0]
    f = torch.from_numpy(f_host).cuda()
    if args.only_apply_b:
        z = mixed.apply_B(f)
        torch.cuda.synchronize()
        for _ in range(args.only_apply_b):
            z = mixed.apply_B(f)
        torch.cuda.synchronize()
        print(json.dumps({"apply_B": args.only_apply_b, "engine": mixed.engine_info(1)}), flush=True)
        return
    plain = S.Precond(sysm, args.nH, S.STARS_ALL, preset["dir_lo"], preset["dir_hi"], precision=S.FP64)
    coarse32 = S.Precond(sysm, args.nH, S.STARS_ALL, preset["dir_lo"], preset["dir_hi"],
                         precision=S.FP32_STARS_COARSE)
    log(f"set up fiber2d_20k H=1/{args.nH}: {sysm.n} dofs, {mixed.nstars} stars")

    # kernel timing legs (eager launches, one iteration per read-back)
    rp_prof = timed_solves(plain, f, max(3, args.steps // 4), 1, args.rtol, profile=True)
    rm_prof = timed_solves(mixed, f, max(3, args.steps // 4), 1, args.rtol, profile=True)
    # timed legs: graph replay (the product configuration), and eager launches
    rm = timed_solves(mixed, f, args.steps, args.warmup, args.rtol, use_graph=True)
    rp = timed_solves(plain, f, args.steps, args.warmup, args.rtol, use_graph=True)
    rc = timed_solves(coarse32, f, args.steps, args.warmup, args.rtol, use_graph=True)
    rme = timed_solves(mixed, f, args.steps, args.warmup, args.rtol)
    rpe = timed_solves(plain, f, args.steps, args.warmup, args.rtol)
    log("headline legs done")

    multi = {}
    for k in (8, 16):
        F = torch.from_numpy(W.rhs(sysm.n, k, seed=17)).cuda()
        for name, pre in (("mixed", mixed), ("plain", plain)):
            r = timed_solves(pre, F, max(2, args.steps // 4), 1, args.rtol, use_graph=True)
            n_solves = k * max(2, args.steps // 4)
            multi[f"{name}_k{k}"] = {"solves_per_s": round(n_solves / r["total_s"], 2),
                                     "ms_per_batch": round(r["total_s"] / max(2, args.steps // 4) * 1e3, 3),
                                     "max_iterations": int(max(i["iters"] for i in r["info"])),
                                     "max_res_true": max(i["res_true"] for i in r["info"])}
    log("multi-RHS legs done")

    # the mesh-size sweep of the same network (H = 1/16, 1/32, 1/64)
    h_sweep = {}
    if not args.no_h_sweep:
        for nH in (16, 32, 64):
            row = {}
            for name, prec in (("mixed", S.FP32_STARS), ("plain", S.FP64)):
                pre = S.Precond(sysm, nH, S.STARS_ALL, preset["dir_lo"], preset["dir_hi"], precision=prec)
                r = timed_solves(pre, f, max(3, args.steps // 4), 1, args.rtol, use_graph=True)
                row[name] = {"solves_per_s": round(max(3, args.steps // 4) / r["total_s"], 2),
                             "iterations": int(r["iters"][-1]), "res_true": r["info"][0]["res_true"],
                             "local_solves_us": pre.engine_info(1)["star_sweep_us"],
                             "stars_supernodal": pre.engine_info(1)["star_sn"],
                             "stars_two_chain": pre.engine_info(1)["star_twins"]}
                row["stars"], row["m0"] = pre.nstars, pre.m0
                row["max_star_dofs"] = pre.factor_info()["max_star_dofs"]
                del pre
            h_sweep[f"H=1/{nH}"] = row
        log("mesh-size sweep done")

    value = args.steps / rm["total_s"]
    plain_value = args.steps / rp["total_s"]
    fim, fip = mixed.factor_info(), plain.factor_info()

    def roof(pre, st):
        ei = pre.engine_info(1)
        dur_s = st["sweep_ms"] / max(st["sweep_launches"], 1) / 1e3
        ach = ei["sweep_bytes"] / dur_s / 1e9
        return dict(bound="hbm", achieved=round(ach, 1), peak=PEAK_HBM_GBS, unit="GB/s",
                    frac=round(ach / PEAK_HBM_GBS, 4), bytes_per_launch=ei["sweep_bytes"],
                    avg_launch_us=round(dur_s * 1e6, 2), launches=st["sweep_launches"], tuning=ei)

    roof_m, roof_p = roof(mixed, rm_prof["stats"]), roof(plain, rp_prof["stats"])
    traffic = None
    if os.path.exists(args.traffic):
        try:
            with open(args.traffic) as fh:
                t = json.load(fh)
            if t.get("bytes_per_launch") == roof_m["bytes_per_launch"] and t.get("kernel_src") == kernel_source_hash():
                traffic = t.get("hbm_bytes_per_launch")
        except Exception:
            traffic = None
    roof_m["traffic"] = traffic
    roof_m["kernel"] = ("local solves (all launches of one application of B: k_star band sweeps, FP32 envelope "
                        "factors, and k_sn supernodal solves for the stars the tuner gives them)")
    roof_m["bytes_basis"] = ("structural non-zeros of each star's factor in the order its kernel uses (RCM for the "
                             "band sweeps, read by both sweeps; minimum degree for the supernodal solves, read once), "
                             "x 4 B, plus 16 B per position (dof index, FP64 gather of r, FP32 slot write)")
    sc = rm_prof["stats"]
    if sc and sc.get("coarse_launches"):
        cus = sc["coarse_ms"] / sc["coarse_launches"] * 1e3
        roof_m["coarse_product_us"] = round(cus, 2)

    u_m = rm["u"].cpu().numpy()
    u_p = rp["u"].cpu().numpy()
    out = {
        "metric": "PCG solves/s at rtol 1e-8 (FP32-star batched vs FP64 plain) + p50/p99 latency",
        "value": round(value, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(rm["total_s"] / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32/f64",
        "data": "synthetic",
        "config": {
            "workload": f"fiber2d_20k_H{args.nH}", "launch": "captured HIP graphs of 2^i iterations",
            "dim": 2, "n_segments": preset["n_segments"], "length": preset["length"], "nH": args.nH,
            "nodes": net.n_nodes, "dofs": sysm.n, "nnz": sysm.nnz, "stars": mixed.nstars, "m0": mixed.m0,
            "rtol": args.rtol, "rhs_per_solve": 1,
            "precision": "FP32 local factors and solves (FP32 accumulation), FP64 coarse operator, FP64 CG "
                         "recurrences, dots and residual checks",
        },
        "latency_ms": {"p50": round(percentile(rm["lat_ms"], 0.5), 3),
                       "p99": round(percentile(rm["lat_ms"], 0.99), 3)},
        "iterations": int(statistics.median(rm["iters"])),
        "iterations_per_s": round(sum(rm["iters"]) / rm["total_s"], 1),
        "res_true": rm["info"][0]["res_true"],
        "plain_fp64": {"value": round(plain_value, 3), "unit": "solves/s",
                       "latency_ms": {"p50": round(percentile(rp["lat_ms"], 0.5), 3),
                                      "p99": round(percentile(rp["lat_ms"], 0.99), 3)},
                       "iterations": int(statistics.median(rp["iters"])), "res_true": rp["info"][0]["res_true"],
                       "roofline_local_solves": roof_p},
        "mixed_over_plain": round(value / plain_value, 3),
        "fp32_coarse_variant": {"value": round(args.steps / rc["total_s"], 3), "unit": "solves/s",
                                "coarse_precision": coarse32.factor_info()["coarse_precision"],
                                "note": "FP32 local solves and the coarse inverse stored in FP32 (FP64 accumulation)"},
        "eager_launches": {"mixed": round(args.steps / rme["total_s"], 3), "plain": round(args.steps / rpe["total_s"], 3)},
        "multi_rhs": multi,
        "h_sweep": h_sweep,
        "roofline": roof_m,
        "setup_s": round(t_setup, 2),
        "factor_info": {"mixed": {k: fim[k] for k in ("star_factor_nnz", "star_rcm_nnz", "star_envelope",
                                                     "star_stored", "star_blob_bytes", "star_index_bytes",
                                                     "sweep_bytes", "sweep_bytes_sn", "max_levels", "max_band",
                                                     "max_star_dofs", "factor_seconds", "coarse_bytes")}},
    }

    if not args.no_configs:
        for name, leg in (("c1", c1_leg), ("c3", c3_leg), ("c4", c4_leg), ("f1", f1_leg), ("f2", f2_leg),
                         ("f4", f4_leg)):
            try:
                out[name] = leg(S, W, torch, args.steps) if name[0] == "c" else leg(S, W, torch)
            except Exception as ex:  # report, keep the other legs
                out[name] = {"error": str(ex)}
            log(f"{name} leg done")

    if not args.no_serving:
        out["serving"] = serving_leg(args.serving_requests, args.serving_rate)
        log("serving leg done")

    if not args.no_cpu_baseline:
        sys.path.insert(0, os.path.join(ROOT, "oracle"))
        import oracle as O
        O.build()
        threads = max(1, min(16, os.cpu_count() or 1))
        u_o, it_o, t1, many_rate, tn, md_nnz = cpu_oracle_leg(O, W, seg, tol, preset, args.nH, f_host, args.rtol,
                                                              threads)
        out["cpu_baseline"] = {"value": round(many_rate, 4), "unit": "solves/s", "cores": threads, "kind": "oracle",
                               "sample": f"{threads} full FP64 oracle PCG solves of the same network with other "
                                         f"right-hand sides, one per core at once ({tn:.1f} s; setup untimed)",
                               "one_core": {"value": round(1.0 / t1, 4), "cores": 1,
                                            "sample": f"one oracle solve of the benchmark right-hand side "
                                                      f"({it_o} iterations, {t1:.1f} s)"}}
        nrm = np.linalg.norm(u_o)
        out["err_vs_oracle"] = {"mixed": float(np.linalg.norm(u_m - u_o) / nrm),
                                "plain": float(np.linalg.norm(u_p - u_o) / nrm), "oracle_iterations": it_o}
        npos = mixed.star_total
        out["roofline"]["md_reference"] = {
            "oracle_min_degree_nnz": md_nnz,
            "ratio_credited_to_md": round((roof_m["bytes_per_launch"] - 16 * npos) / (4 * md_nnz), 3),
            "bytes_if_md_factor_read_once": md_nnz * 4 + 16 * npos,
            "frac_on_md_bytes": round((md_nnz * 4 + 16 * npos) / (roof_m["avg_launch_us"] * 1e-6) / 1e9 /
                                      PEAK_HBM_GBS, 4)}
        log("cpu baseline done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
