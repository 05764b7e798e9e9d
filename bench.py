#!/usr/bin/env python3
"""Single-source SSSP throughput of the MLMQ library on one MI355X.

One step = one complete single-source solve (init + persistent MLMQ kernel)
on a graph already resident in HBM. The headline workload is RMAT scale 23
(edge factor 16, symmetrised, ~258.7M directed edges, source = highest-degree
vertex); the road-like 2048x2048 grid (p_drop 0.05, source = centre) is
measured in the same run. Inputs are seeded synthetic graphs.

Prints one JSON line (see the repository's benchmark contract). GTEPS =
directed edges leaving reachable vertices / solve time. The roofline entry
prices the persistent kernel's algorithmic bytes, 12 B per reachable edge +
32 B per reachable vertex + 4 B per vertex, against 8 TB/s of HBM3E.
The CPU baseline is the oracle (binary-heap Dijkstra, one core) on the same
graph; its output also verifies the GPU distances.
"""
import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import graphgen as gg  # noqa: E402

METRIC = "GTEPS single-source (RMAT-23, grid); batched queries/s + p99 latency vs plain"
HBM_PEAK_GBS = 8000.0
INF = 0xFFFFFFFF


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name):
    if name == "rmat23":
        g = gg.rmat(23, 16, seed=1)
        return g, gg.max_degree_vertex(g), "RMAT scale 23, ef 16, (0.57,0.19,0.19,0.05), symmetrised, w in [1,255]"
    if name == "rmat20":
        g = gg.rmat(20, 16, seed=1)
        return g, gg.max_degree_vertex(g), "RMAT scale 20, ef 16, symmetrised, w in [1,255]"
    if name == "grid2048":
        g = gg.grid(2048, 2048, 0.05, seed=1)
        return g, 1024 * 2048 + 1024, "2048x2048 grid, p_drop 0.05, w in [1,255], source = centre"
    if name == "grid256":
        g = gg.grid(256, 256, 0.0, seed=1)
        return g, 0, "256x256 grid, w in [1,255], source 0"
    raise SystemExit(f"unknown workload {name}")


KERNEL_SRC = os.path.join(ROOT, "paper_2602_10080_amd", "csrc", "mlmq_kernels.hip")


def measured_traffic(workload):
    """HBM bytes per launch of the persistent kernel from the committed
    rocprofv3 counter summary for this workload (FETCH_SIZE + WRITE_SIZE, each
    scaled by the same counter's reading for a copy of known size), or None if
    there is none or the kernel source changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_mlmq_worker_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    if rec.get("kernel_sha256") != sha:
        return None
    return rec


def roofline(p):
    """The roofline record of the persistent kernel on workload summary p:
    algorithmic bytes per launch / its HIP-event duration against 8 TB/s, and,
    when the committed counter summary matches the kernel source, the memory
    traffic per launch: FETCH_SIZE and WRITE_SIZE scaled by a copy of known
    size (traffic), the DRAM-bound 32-byte read sectors (calibrated 1.00 on
    the copy) and what that traffic is per second of the solve."""
    rec = measured_traffic(p["workload"])
    out = {"bound": "hbm", "achieved": p["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": p["achieved_gbs"] / HBM_PEAK_GBS, "traffic": None}
    if rec:
        t = rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
        out["traffic"] = t
        out["traffic_vs_algorithmic"] = t / p["algorithmic_bytes"]
        out["traffic_gbs"] = t / (p["worker_ms"] * 1e-3) / 1e9
        out["traffic_frac"] = out["traffic_gbs"] / HBM_PEAK_GBS
        if "dram_read_bytes_per_launch" in rec:
            out["dram_read_bytes"] = rec["dram_read_bytes_per_launch"]
        out["traffic_note"] = ("L2-to-memory requests; they include lines the 256 MB Infinity Cache serves, "
                               "so this bounds HBM traffic from above")
    return out


def reach(csr, dist):
    fin = dist != INF
    return int(fin.sum()), int(csr.degrees()[fin].sum())


def measure(mlmq, torch, csr, src, overrides, steps, warmup, bare=False):
    g = mlmq.Graph.from_csr(csr)
    cfg = g.config()
    for k, v in (json.loads(overrides) if overrides else {}).items():
        setattr(cfg, k, int(v))
    out = mlmq.new_dist(csr.n)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        mlmq.sssp(g, src, out=out, config=cfg, stream=stream)
    torch.cuda.synchronize()
    walls, kms, wms, last = [], [], [], None
    t_all = time.perf_counter()
    for _ in range(steps):
        t0 = time.perf_counter()
        _, st = mlmq.sssp(g, src, out=out, config=cfg, stream=stream, stats=True)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        kms.append(st["kernel_ms"])
        wms.append(st["worker_ms"])
        last = st
    total = time.perf_counter() - t_all
    if bare:
        dist = mlmq.to_numpy(out)
        g.close()
        return dict(walls=walls, kernel_ms=kms, worker_ms=wms, stats=last, dist=dist, total=total, cfg=cfg,
                    host_output_ms=None, check_violations=None, single_pass_ms=None)
    # the same solve into a host buffer: the library copies the distances back
    # (PCIe-inclusive time; never the headline value)
    host_out = np.empty(csr.n, np.uint32)
    host_ms = []
    for _ in range(3):
        t0 = time.perf_counter()
        mlmq.sssp(g, src, out=host_out, config=cfg, stream=stream)
        host_ms.append((time.perf_counter() - t0) * 1e3)
    # device optimality check of the output; its edge pass (every edge word and
    # both labels read once) is the cost of one relaxation sweep of the graph
    viol, pass_ms = None, []
    try:
        for _ in range(4):
            viol, ms = mlmq.check(g, src, out, stream=stream)
            pass_ms.append(ms)
    except mlmq.MlmqError as e:
        log(f"[bench] device check unavailable: {e}")
    dist = mlmq.to_numpy(out)
    g.close()
    if not np.array_equal(host_out, dist):
        raise SystemExit("host-output solve differs from the device-output solve")
    return dict(walls=walls, kernel_ms=kms, worker_ms=wms, stats=last, dist=dist, total=total, cfg=cfg,
                host_output_ms=statistics.median(host_ms),
                check_violations=viol, single_pass_ms=statistics.median(pass_ms[1:]) if pass_ms else None)


def summarize(name, desc, csr, src, res, cfg):
    n_reach, m_reach = reach(csr, res["dist"])
    wall_ms = statistics.median(res["walls"]) * 1e3
    k_ms = statistics.median(res["kernel_ms"])
    w_ms = statistics.mean(res["worker_ms"])
    abytes = 12 * m_reach + 32 * n_reach + 4 * csr.n
    st = res["stats"]
    sp = res["single_pass_ms"]
    return dict(
        workload=name, description=desc, n=csr.n, m=csr.m, source=int(src), n_reach=n_reach, m_reach=m_reach,
        ms_per_step=wall_ms, kernel_ms=k_ms, worker_ms=w_ms,
        gteps=m_reach / (wall_ms * 1e-3) / 1e9, gteps_device=m_reach / (k_ms * 1e-3) / 1e9,
        gteps_undirected=m_reach / 2 / (wall_ms * 1e-3) / 1e9,
        ms_host_output=res["host_output_ms"],
        algorithmic_bytes=abytes, achieved_gbs=abytes / (w_ms * 1e-3) / 1e9,
        work_ratio=st["expansions"] / max(n_reach, 1), edges_scanned=st["edges"], pushes=st["pushes"],
        l2_blocks=st["l2_writes"], hub_chunks=st["hub_chunks"], grid_wgs=st["grid_wgs"],
        config=cfg.as_dict(), device_check_violations=res["check_violations"],
        single_pass_ms=sp, single_pass_gedges=(csr.m / sp / 1e6) if sp else None,
        scan_gedges=st["edges"] / w_ms / 1e6,
        scan_vs_single_pass=(st["edges"] / w_ms) / (csr.m / sp) if sp else None,
    )


def bench_bfs(mlmq, torch, csr, src, steps=5):
    """Breadth-first levels on the same queues (same graph, same source)."""
    g = mlmq.Graph.from_csr(csr)
    out = mlmq.new_dist(csr.n)
    mlmq.bfs(g, src, out=out)
    torch.cuda.synchronize()
    wms = []
    for _ in range(steps):
        _, st = mlmq.bfs(g, src, out=out, stats=True)
        wms.append(st["worker_ms"])
    torch.cuda.synchronize()
    lv = mlmq.to_numpy(out)
    n_reach, m_reach = reach(csr, lv)
    g.close()
    w = statistics.median(wms)
    levels = int(lv[lv != INF].max()) + 1
    log(f"[bench] bfs: {w:.2f} ms, {m_reach / w / 1e6:.2f} GTEPS, {levels} levels, {w / levels * 1e3:.2f} us per level")
    return dict(worker_ms=w, gteps_device=m_reach / w / 1e6, work_ratio=st["expansions"] / max(1, n_reach),
                levels=levels, us_per_level=w / levels * 1e3)


def stream_probe(torch, nbytes=1 << 30, reps=5):
    """Achievable device bandwidth: a plain 1 GiB device-to-device copy (one
    read and one write of every byte), timed with events on the stream."""
    src = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        dst.copy_(src)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2 * nbytes / ms / 1e6


def cpu_baseline(csr, src, gpu_dist, max_seconds=30.0):
    """Oracle Dijkstra on one core; repeated while under the time bound."""
    import oracle
    times, want = [], None
    while not times or (sum(times) < max_seconds / 3 and len(times) < 3):
        t0 = time.perf_counter()
        want = oracle.dijkstra(csr, src)
        times.append(time.perf_counter() - t0)
    _, m_reach = reach(csr, want)
    t = statistics.median(times)
    # the oracle's certificate of the GPU vector also gives the fewest-hop
    # depth of the shortest-path DAG (for the latency floor)
    code, _, depth = oracle.certificate(csr, src, gpu_dist)
    return dict(value=m_reach / t / 1e9, unit="GTEPS", cores=1, kind="oracle",
                sample=f"{len(times)} full single-source solve(s), median {t:.2f} s",
                seconds=t, sp_depth=int(depth) if code == 0 else None), bool(np.array_equal(want, gpu_dist))


def host_info():
    """Host CPU of this box: logical CPUs the OS reports, the model name, and
    the worker threads a CPU baseline uses (the host share of one GPU: at most
    16 threads)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    nproc = os.cpu_count() or 1
    return dict(nproc=nproc, cpu_model=model, threads=min(16, nproc))


def oracle_pool(csrs, srcs, gpu_out, what, max_seconds=None):
    """The oracle over a thread pool (one query per thread; the C oracle
    releases the GIL), timed as a throughput baseline. Every finished query is
    compared with the GPU's vector (gpu_out(i), a host array). With max_seconds, queries are submitted in
    order until the time bound is reached (a bounded sample)."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    hi = host_info()
    done, equal = 0, True
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=hi["threads"]) as ex:
        futs = []
        for i in range(len(srcs)):
            if max_seconds is not None and time.perf_counter() - t0 > max_seconds:
                break
            futs.append((i, ex.submit(oracle.dijkstra, csrs[i], srcs[i])))
            if max_seconds is not None and len(futs) >= hi["threads"]:
                # keep at most one round of queries in flight so the bound holds
                j, f = futs.pop(0)
                equal = equal and bool(np.array_equal(f.result(), gpu_out(j)))
                done += 1
        for j, f in futs:
            equal = equal and bool(np.array_equal(f.result(), gpu_out(j)))
            done += 1
    t = time.perf_counter() - t0
    cpu = dict(value=done / t, unit="queries/s", cores=hi["threads"], kind="oracle",
               sample=f"{done} of {what}, one query per thread, {t:.1f} s", host=hi)
    return cpu, equal


def bench_batch(mlmq, torch, tune_ms, nrmat=256, ngrid=64):
    """Many queries in one persistent launch vs the same queries as sequential
    plain solves (graphs resident, autotuned config per graph for both)."""
    rmat = gg.rmat(20, 16, seed=1)
    grid = gg.grid(1024, 1024, 0.05, seed=1)
    gr, gd = mlmq.Graph.from_csr(rmat), mlmq.Graph.from_csr(grid)
    t0 = time.perf_counter()
    cr = mlmq.autotune(gr, tune_ms)
    cd = mlmq.autotune(gd, tune_ms)
    log(f"[bench] batch: autotuned in {time.perf_counter() - t0:.1f}s")
    srcs = [int(x) for x in gg.sample_sources(rmat, nrmat, seed=2)] + \
           [int(x) for x in gg.sample_sources(grid, ngrid, seed=3)]
    graphs = [gr] * nrmat + [gd] * ngrid
    cfgs = [cr] * nrmat + [cd] * ngrid
    csrs = [rmat] * nrmat + [grid] * ngrid
    outs = [mlmq.new_dist(c.n) for c in csrs]
    seq = [mlmq.new_dist(c.n) for c in csrs]
    stream = torch.cuda.current_stream()
    mlmq.sssp_batch(graphs, srcs, outs=outs, configs=cfgs, stream=stream)  # warm-up (captures the launch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, status = mlmq.sssp_batch(graphs, srcs, outs=outs, configs=cfgs, stream=stream)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    for g, s, o, c in zip(graphs[:4], srcs[:4], seq[:4], cfgs[:4]):  # warm-up
        mlmq.sssp(g, s, out=o, config=c, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g, s, o, c in zip(graphs, srcs, seq, cfgs):
        mlmq.sssp(g, s, out=o, config=c, stream=stream)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    same = all(torch.equal(a, b) for a, b in zip(outs, seq))
    nq = nrmat + ngrid
    # CPU baseline: the oracle, one query per thread over the host's CPU share
    # for one GPU, on every query of the batch; its vectors also check every
    # batched output element by element
    cpu, exact = oracle_pool(csrs, srcs, lambda i: mlmq.to_numpy(outs[i]),
                             f"all {nq} queries of the batch ({nrmat} RMAT-20, {ngrid} grid1024)")
    res = dict(queries=nq, cpu_baseline=cpu, workload=f"{nrmat} sources RMAT-20 + {ngrid} sources grid1024 p0.05",
               batch_s=t_batch, sequential_s=t_seq, batch_qps=nq / t_batch, sequential_qps=nq / t_seq,
               speedup=t_seq / t_batch, statuses_ok=all(x == 0 for x in status),
               batch_equals_sequential=same, oracle_checked=nq, oracle_equal=exact,
               tuned={"rmat20": cr.as_dict(), "grid1024": cd.as_dict()})
    log(f"[bench] batch: {nq} queries {t_batch:.3f}s ({nq / t_batch:.1f} q/s) vs sequential {t_seq:.3f}s "
        f"({nq / t_seq:.1f} q/s), same={same} oracle={exact}")
    for g in (gr, gd):
        g.close()
    return res


def _percentiles(lat):
    a = np.sort(np.asarray(lat))
    return float(np.percentile(a, 50)), float(np.percentile(a, 99))


def bench_serve(mlmq, torch, nreq, load, budget_gb, seed=7, rate=None, legs=("fifo", "server")):
    """Poisson arrivals over five resident graphs, served by the
    continuous-batching server and, on the same trace, by a FIFO loop of plain
    solves. Latency = completion - arrival. rate (q/s) fixes the arrival rate
    (else load x the FIFO service rate measured on the head of the trace);
    legs picks which of the two runs (a long trace may be split over runs)."""
    csrs = [gg.grid(512, 512, 0.05, seed=11), gg.grid(2048, 2048, 0.05, seed=12), gg.rmat(20, 16, seed=13),
            gg.rmat(22, 16, seed=14), gg.uniform(1 << 22, 1 << 25, wmax=65535, seed=15)]
    names = ["grid512", "grid2048", "rmat20", "rmat22", "uniform4M"]
    graphs = [mlmq.Graph.from_csr(c) for c in csrs]
    rng = np.random.default_rng(seed)
    gid = rng.integers(0, len(csrs), nreq)
    src = np.array([rng.integers(0, csrs[g].n) for g in gid])
    stream = torch.cuda.current_stream()
    per_graph = [mlmq.new_dist(c.n) for c in csrs]
    # FIFO service rate, measured on the head of the trace
    probe = min(nreq, 60)
    for i in range(min(5, nreq)):
        mlmq.sssp(graphs[gid[i]], int(src[i]), out=per_graph[gid[i]], stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(probe):
        mlmq.sssp(graphs[gid[i]], int(src[i]), out=per_graph[gid[i]], stream=stream)
    torch.cuda.synchronize()
    mu = probe / (time.perf_counter() - t0)
    lam = rate if rate else load * mu
    arrive = np.cumsum(rng.exponential(1.0 / lam, nreq))
    log(f"[bench] serve: FIFO service rate {mu:.1f} q/s, arrivals at {lam:.1f} q/s "
        f"({'fixed' if rate else str(load) + 'x'})")

    # FIFO loop of plain solves
    fifo_lat, t_start = [], time.perf_counter()
    keep = {}
    for i in range(nreq if "fifo" in legs else 0):
        if i % 500 == 0:
            log(f"[bench] serve: FIFO loop at request {i}")
        now = time.perf_counter() - t_start
        if now < arrive[i]:
            time.sleep(arrive[i] - now)
        g = gid[i]
        mlmq.sssp(graphs[g], int(src[i]), out=per_graph[g], stream=stream)
        torch.cuda.synchronize()
        fifo_lat.append(time.perf_counter() - t_start - arrive[i])
        if i % max(1, nreq // 8) == 0:
            keep[i] = mlmq.to_numpy(per_graph[g]).copy()
    fifo_span = time.perf_counter() - t_start - arrive[0]
    log(f"[bench] serve: FIFO loop done in {fifo_span:.1f}s")
    if "server" not in legs:
        f50, f99 = _percentiles(fifo_lat)
        for g in graphs:
            g.close()
        return dict(requests=nreq, graphs=names, arrival_rate_qps=lam, fifo_service_rate_qps=mu, load=load,
                    fifo_qps=nreq / fifo_span if fifo_lat else None, fifo_p50_ms=f50 * 1e3, fifo_p99_ms=f99 * 1e3, legs=list(legs))

    # continuous-batching server (one output buffer per graph and slot in
    # flight would do; a buffer per request keeps every result for the checks)
    outs = [mlmq.new_dist(csrs[g].n) for g in gid]
    torch.cuda.synchronize()
    srv = mlmq.Server(graphs, mem_budget_bytes=int(budget_gb * (1 << 30)), max_slots=64)
    tickets, sub_ns = [], []
    t_start = time.perf_counter()
    try:
        for i in range(nreq):
            if i % 500 == 0:
                log(f"[bench] serve: server at request {i}")
            now = time.perf_counter() - t_start
            if now < arrive[i]:
                time.sleep(arrive[i] - now)
            tickets.append(srv.submit(int(gid[i]), int(src[i]), outs[i]))
        status = [srv.wait(t, 120000) for t in tickets]
        times = [srv.times(t) for t in tickets]
    finally:
        srv.close()
    t0_ns = times[0][0] - int(arrive[0] * 1e9)
    srv_lat = [(b - t0_ns) / 1e9 - arrive[i] for i, (a, b) in enumerate(times)]
    srv_span = (max(b for _, b in times) - t0_ns) / 1e9 - arrive[0]
    same = all(np.array_equal(mlmq.to_numpy(outs[i]), keep[i]) for i in keep) if keep else None
    # CPU baseline: the oracle on the trace's requests in arrival order, one per
    # thread, for about 20 s; each vector is compared with the served one
    cpu, cpu_equal = oracle_pool([csrs[g] for g in gid], [int(x) for x in src], lambda i: mlmq.to_numpy(outs[i]),
                                 f"the {nreq} requests in arrival order", max_seconds=20.0)
    f50, f99 = _percentiles(fifo_lat) if fifo_lat else (float("nan"), float("nan"))
    s50, s99 = _percentiles(srv_lat)
    res = dict(requests=nreq, graphs=names, arrival_rate_qps=lam, fifo_service_rate_qps=mu, load=load,
               mem_budget_gb=budget_gb,
               server_qps=nreq / srv_span, server_p50_ms=s50 * 1e3, server_p99_ms=s99 * 1e3,
               fifo_qps=nreq / fifo_span if fifo_lat else None, fifo_p50_ms=f50 * 1e3, fifo_p99_ms=f99 * 1e3,
               statuses_ok=all(x == 0 for x in status), served_equals_alone=same, compared=len(keep),
               cpu_baseline=cpu, oracle_equal=cpu_equal)
    log(f"[bench] serve: server {res['server_qps']:.1f} q/s p50 {res['server_p50_ms']:.2f} ms "
        f"p99 {res['server_p99_ms']:.2f} ms | FIFO {res['fifo_qps'] or float('nan'):.1f} q/s "
        f"p50 {res['fifo_p50_ms']:.2f} ms p99 {res['fifo_p99_ms']:.2f} ms | same={same}")
    res["legs"] = list(legs)
    for g in graphs:
        g.close()
    return res


def pq_study(mlmq, torch, reps=3):
    """Section 5's priority-queue case study on synthetic stand-ins: the L2
    priority queue (L2PQ) and the multi-queue (L2MPQ, 16 queues) alone and
    under L0 + L1 queues, at several launch sizes, beside the FIFO and bucket
    L2 under the same L0 + L1. Median device time of the persistent kernel
    and work ratio (expansions / reachable vertices) per point; every output
    is checked by the device optimality check."""
    graphs = {"road512": (gg.grid(512, 512, 0.05, seed=11), 256 * 512 + 256),
              "rmat20": (lambda c: (c, gg.max_degree_vertex(c)))(gg.rmat(20, 16, seed=13))}
    fams = {
        "L2PQ": dict(l0_rows=0, l1_type=0, l2_type=2, pnum=1),
        "L2MPQ16": dict(l0_rows=0, l1_type=0, l2_type=2, pnum=16),
        "L0L1-L2PQ": dict(l0_rows=1, l1_type=2, l2_type=2, pnum=1),
        "L0L1-L2MPQ16": dict(l0_rows=1, l1_type=2, l2_type=2, pnum=16),
        "L0L1-L2V": dict(l0_rows=1, l1_type=2, l2_type=0),
        "L0L1-L2DQ": dict(l0_rows=1, l1_type=2, l2_type=1),
    }
    out = {}
    for gname, (csr, src) in graphs.items():
        g = mlmq.Graph.from_csr(csr)
        base = g.config()
        d = mlmq.new_dist(csr.n)
        rows = []
        for fam, kw in fams.items():
            for waves in (128, 512, 2048):
                cfg = base.copy(**kw, grid_wgs=waves, timeout_ms=20000, th_hub=0)
                ms, st = [], None
                try:
                    for _ in range(reps):
                        _, st = mlmq.sssp(g, src, out=d, config=cfg, stats=True)
                        ms.append(st["worker_ms"])
                    bad, _ = mlmq.check(g, src, d)
                except mlmq.MlmqError as e:
                    rows.append(dict(queues=fam, waves=waves, error=str(e)[:120]))
                    log(f"[bench] pq study {gname} {fam} {waves}: {e}")
                    continue
                n_reach = int((mlmq.to_numpy(d) != INF).sum())
                rows.append(dict(queues=fam, waves=waves, worker_ms=statistics.median(ms),
                                 work_ratio=st["expansions"] / max(1, n_reach), l2_writes=st["l2_writes"],
                                 violations=int(bad)))
                log(f"[bench] pq study {gname} {fam} waves {waves}: {statistics.median(ms):.2f} ms, "
                    f"work {rows[-1]['work_ratio']:.2f}, violations {bad}")
        g.close()
        out[gname] = rows
    return out


# ------------------------------------------------------------ counter summaries

COUNTER_PASSES = {
    # pass name: counters (each pass fits the per-block limits of one rocprofv3 run)
    "fetch": ["FETCH_SIZE"],
    "write": ["WRITE_SIZE", "TCC_EA0_WRREQ_DRAM_sum"],
    "dram": ["TCC_EA0_RDREQ_DRAM_32B_sum", "TCC_EA0_RDREQ_DRAM_sum", "TCC_EA0_WRREQ_ATOMIC_DRAM_32B_sum",
             "TCC_EA0_ATOMIC_sum"],
    "cache": ["TCC_HIT_sum", "TCC_MISS_sum", "SQ_INSTS_LDS", "SQ_LDS_BANK_CONFLICT", "SQ_WAVE_CYCLES",
              "SQ_BUSY_CYCLES", "SQ_WAIT_INST_ANY"],
    # instruction issue: how much of a wave's life is spent issuing, and what
    "issue": ["SQ_WAVES", "SQ_WAVE_CYCLES", "SQ_WAIT_ANY", "SQ_ACTIVE_INST_ANY", "SQ_INSTS_VALU", "SQ_INSTS_SALU",
              "SQ_INSTS_VMEM", "SQ_INSTS_SMEM"],
    "issue2": ["SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_SCA", "SQ_ACTIVE_INST_LDS", "SQ_ACTIVE_INST_VMEM",
               "SQ_INSTS_BRANCH", "SQ_INSTS_LDS", "SQ_WAIT_INST_LDS", "SQ_WAVE_CYCLES"],
    # instruction and scalar data caches
    "icache": ["SQC_ICACHE_REQ", "SQC_ICACHE_HITS", "SQC_ICACHE_MISSES", "SQC_ICACHE_MISSES_DUPLICATE",
               "SQC_DCACHE_REQ", "SQC_DCACHE_HITS", "SQC_DCACHE_MISSES", "SQC_TC_INST_REQ"],
}


def _counter_rows(path):
    """{dispatch id: (kernel name, {counter: value})} from a rocprofv3 counter CSV."""
    import csv
    out = {}
    with open(path) as fh:
        for r in csv.DictReader(fh):
            d = out.setdefault(int(r["Dispatch_Id"]), [r["Kernel_Name"], {}])
            d[1][r["Counter_Name"]] = d[1].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return out


def summarize_counters(root, workloads, warmup, steps):
    """Per-launch counter values of the persistent kernel from the counter
    passes under root/<pass>/ (run with --bare, so each workload contributes
    warmup + steps launches in order), the copy calibration from
    root/copy_<pass>/, and the traffic record per workload."""
    import glob
    import hashlib
    per = {w: {} for w in workloads}
    calib = {}
    for pas in COUNTER_PASSES:
        f = glob.glob(os.path.join(root, pas, "**", "*counter_collection.csv"), recursive=True)
        if f:
            rows = _counter_rows(f[0])
            launches = [v for _, v in sorted(rows.items()) if "mlmq_worker" in v[0]]
            k = warmup + steps
            if len(launches) != k * len(workloads):
                raise SystemExit(f"{pas}: {len(launches)} worker launches, expected {k * len(workloads)}")
            for i, w in enumerate(workloads):
                timed = launches[i * k + warmup:(i + 1) * k]
                for c in timed[0][1]:
                    per[w][c] = statistics.mean(t[1][c] for t in timed)
        f = glob.glob(os.path.join(root, "copy_" + pas, "**", "*counter_collection.csv"), recursive=True)
        if f:
            rows = _counter_rows(f[0])
            cp = [v for _, v in sorted(rows.items()) if "copyBuffer" in v[0]]
            big = [v for v in cp if v[1].get(COUNTER_PASSES[pas][0], 0) > 0]
            for c in big[-1][1]:
                calib[c] = statistics.mean(v[1][c] for v in big[-3:])
    sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    copy_kib = 1 << 20  # the copy probe moves 1 GiB each way
    out = {}
    for w, c in per.items():
        if "FETCH_SIZE" not in c or "WRITE_SIZE" not in c:
            continue
        fs = copy_kib / calib["FETCH_SIZE"] if "FETCH_SIZE" in calib else 1.0
        ws = copy_kib / calib["WRITE_SIZE"] if "WRITE_SIZE" in calib else 1.0
        rec = dict(kernel="mlmq::mlmq_worker", workload=w, kernel_sha256=sha, launches_averaged=steps,
                   raw_fetch_kib_per_launch=c["FETCH_SIZE"], raw_write_kib_per_launch=c["WRITE_SIZE"],
                   fetch_scale=fs, write_scale=ws,
                   fetch_bytes_per_launch=c["FETCH_SIZE"] * 1024 * fs,
                   write_bytes_per_launch=c["WRITE_SIZE"] * 1024 * ws,
                   counters_per_launch=c, copy_calibration=calib)
        if "TCC_EA0_RDREQ_DRAM_32B_sum" in c:
            rec["dram_read_bytes_per_launch"] = c["TCC_EA0_RDREQ_DRAM_32B_sum"] * 32
        out[w] = rec
        with open(os.path.join(ROOT, "profiles", f"traffic_mlmq_worker_{w}.json"), "w") as fh:
            json.dump(rec, fh, indent=1)
    print(json.dumps({w: {k: v for k, v in r.items() if k not in ("counters_per_launch", "copy_calibration")}
                      for w, r in out.items()}, indent=1))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rmat23")
    ap.add_argument("--also", default="grid2048,grid256", help="comma-separated extra workloads ('' for none)")
    ap.add_argument("--config", default="", help="JSON overrides of the queue config (primary workload)")
    ap.add_argument("--also-config", default="", help="JSON overrides for the extra workloads")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch", type=int, default=1, help="run the batched-form comparison (0/1)")
    ap.add_argument("--tune-ms", type=int, default=3000, help="autotuner budget per graph (batch)")
    ap.add_argument("--serve", type=int, default=2000, help="serving requests (0 = skip)")
    ap.add_argument("--serve-load", type=float, default=1.5, help="arrival rate / FIFO service rate")
    ap.add_argument("--serve-budget-gb", type=float, default=8.0)
    ap.add_argument("--serve-rate", type=float, default=0.0, help="fixed arrival rate in q/s (0 = load x FIFO rate)")
    ap.add_argument("--serve-legs", default="fifo,server", help="which serving runs: fifo, server or both")
    ap.add_argument("--bare", action="store_true",
                    help="only the warm-up and timed solves of each workload (for counter passes)")
    ap.add_argument("--summarize-counters", default="",
                    help="directory of rocprofv3 counter passes: write profiles/traffic_mlmq_worker_<w>.json and exit")
    ap.add_argument("--pq-study", action="store_true",
                    help="also run the priority-queue case study (road512, rmat20) into the detail section")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB three times (calibrates HBM counters)")
    args = ap.parse_args()
    if args.summarize_counters:
        workloads = [args.workload] + [w for w in args.also.split(",") if w]
        summarize_counters(args.summarize_counters, workloads, args.warmup, args.steps)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the single-source solve runs on one device)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2602_10080_amd as mlmq
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    torch.cuda.set_device(0)

    if args.copy_probe_mib:
        nbytes = args.copy_probe_mib << 20
        src = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": nbytes, "copy_probe_bytes_written": nbytes, "launches": 3}))
        return

    results = {}
    primary = None
    for i, name in enumerate([args.workload] + [w for w in args.also.split(",") if w]):
        t0 = time.perf_counter()
        csr, src, desc = make_workload(name)
        log(f"[bench] {name}: n={csr.n} m={csr.m} generated in {time.perf_counter() - t0:.1f}s")
        res = measure(mlmq, torch, csr, src, args.config if i == 0 else args.also_config, args.steps,
                      args.warmup, bare=args.bare)
        s = summarize(name, desc, csr, src, res, res["cfg"])
        log(f"[bench] {name}: {s['ms_per_step']:.3f} ms/step wall, kernel {s['kernel_ms']:.3f} ms, "
            f"{s['gteps']:.2f} GTEPS, work ratio {s['work_ratio']:.2f}")
        if s["single_pass_ms"]:
            log(f"[bench] {name}: device check {s['device_check_violations']} violations; one sweep of all edges "
                f"{s['single_pass_ms']:.3f} ms ({s['single_pass_gedges']:.1f} G edges/s), solve scans "
                f"{s['scan_gedges']:.1f} G edges/s = {s['scan_vs_single_pass']:.2f} of that")
        if args.bare:
            results[name] = s
            if i == 0:
                primary = s
            continue
        if not args.no_cpu_baseline:
            cb, ok = cpu_baseline(csr, src, res["dist"])
            s["cpu_baseline"] = cb
            s["verified_against_oracle"] = ok
            log(f"[bench] {name}: oracle {cb['seconds']:.2f} s ({cb['value']:.4f} GTEPS), match={ok}")
        if name in ("rmat23", "grid2048", "grid256"):
            s["bfs"] = bench_bfs(mlmq, torch, csr, src)
            depth = s.get("cpu_baseline", {}).get("sp_depth")
            if depth is not None and name.startswith("grid"):
                # latency floors of a high-diameter graph (on power-law graphs a
                # level is throughput-bound, not a round trip, and no floor is
                # given): the fewest-hop depth of the shortest-path DAG times
                # (a) the time of one dependent relaxation hop (row bounds, edge
                # word, atomicMin, each waiting for the previous) measured by a
                # probe kernel with no queue at all, independent of the solver;
                # (b) the per-level time of the breadth-first run on the same
                # queues (the solver's own round trip per level)
                g = mlmq.Graph.from_csr(csr)
                hop_ns, hand_ns = mlmq.latency_probe(g, src, 8192)
                g.close()
                floor = (depth + 1) * hop_ns / 1e6
                bfs_floor = (depth + 1) * s["bfs"]["us_per_level"] / 1e3
                s["sp_depth"] = int(depth)
                s["hop_probe_ns"] = hop_ns
                s["handoff_probe_ns"] = hand_ns
                s["latency_floor_ms"] = floor
                s["vs_latency_floor"] = s["worker_ms"] / floor
                s["bfs_level_floor_ms"] = bfs_floor
                s["vs_bfs_level_floor"] = s["worker_ms"] / bfs_floor
                log(f"[bench] {name}: shortest-path depth {depth} hops; dependent hop {hop_ns:.0f} ns, "
                    f"hand-off {hand_ns:.0f} ns; latency floor {floor:.2f} ms (solve = {s['vs_latency_floor']:.2f} x); "
                    f"breadth-first level floor {bfs_floor:.2f} ms (solve = {s['vs_bfs_level_floor']:.2f} x)")
        results[name] = s
        if i == 0:
            primary = s
        del csr, res

    if args.bare:
        print(json.dumps({k: {kk: v[kk] for kk in ("workload", "ms_per_step", "worker_ms", "gteps")}
                          for k, v in results.items()}), flush=True)
        return
    stream_gbs = stream_probe(torch)
    log(f"[bench] stream probe (1 GiB device copy): {stream_gbs:.0f} GB/s")
    for s in results.values():
        s["achieved_vs_stream"] = s["achieved_gbs"] / stream_gbs
    batch = bench_batch(mlmq, torch, args.tune_ms) if args.batch else None
    serving = bench_serve(mlmq, torch, args.serve, args.serve_load, args.serve_budget_gb, rate=args.serve_rate or None,
                          legs=tuple(args.serve_legs.split(","))) if args.serve else None
    pq = pq_study(mlmq, torch) if args.pq_study else None

    p = primary
    line = {
        "metric": METRIC,
        "value": p["gteps"],
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": p["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": p["workload"], "graph": p["description"], "n": p["n"], "m": p["m"],
                   "source": p["source"], "queues": p["config"]},
        "roofline": roofline(p),
        "cpu_baseline": p.get("cpu_baseline"),
        "verified_against_oracle": p.get("verified_against_oracle"),
        "device_check_violations": p.get("device_check_violations"),
        "stream_probe": {"gbs": stream_gbs, "what": "1 GiB device-to-device copy, read + write bytes / event time"},
        "batch": batch,
        "serving": serving,
        "detail": {k: {kk: vv for kk, vv in v.items() if kk not in ("config",)} for k, v in results.items()},
    }
    if pq is not None:
        line["pq_case_study"] = pq
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
