#!/usr/bin/env python3
"""Benchmark: triangle counting + truss decomposition edges/s on one MI355X.

One step = the whole hot path on one synthetic graph whose raw pairs are
already in HBM: gc_build_csr (normalise, degree order, oriented CSR, in-edge
index) + gc_triangle_count + gc_truss_decomposition (support counted once,
then edges peeled level by level with incremental support updates).
value = m / step time, m = undirected edges after normalisation (the rate of
Sec. IV-B: edges over execution time, file reading excluded).

Also reported (one JSON line, rank 0):
  roofline      the dominant triangle-count kernel (the longest degree-bin
                launch) against HBM peak: its own algorithmic bytes (the
                tail model of the schedule) / its kernel time (HIP events around
                the launch on the stream it runs on), with its counter-measured
                HBM bytes per launch beside it; the whole pass, and the
                whole-list model B_TC = min(16n+20m+4 S_dst, 16n+24m+4 S_src)
                as context;
  cpu_baseline  the CPU oracle timed on the host: one thread on a bounded
                sample (a smaller R-MAT of the same family), and the count
                over every host core at R-MAT scale 20, with the CPU model;
  phases        build / count / decomposition times;
  batch, serve  the batched and serving paths against one graph per call.

Usage: python bench.py [--steps K] [--warmup W] [--scale 24] [--workload rmat|er]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def gen_inputs(workload: str, scale: int, ef: int, seed: int):
    import graphgen as gg
    if workload == "rmat":
        return gg.rmat(scale, ef, seed=seed)
    if workload == "er":
        n = 1 << scale
        return gg.er(n, ef * n, seed=seed)
    raise ValueError(workload)


class EnergyMeter:
    """GPU energy over a region, read through amdsmi (read-only telemetry) on
    the device matched to torch's by PCI bus: the accumulating energy counter
    if it advances over the region, else socket power sampled every 5 ms and
    integrated.  If neither is available stop() returns None and `source`
    says why."""

    def __init__(self, torch, dev):
        import threading
        self.h = None
        self.source = "amdsmi"
        self.samples = []
        self.stop_ev = threading.Event()
        self.th = threading.Thread(target=self._sample, daemon=True)
        try:
            import amdsmi
            self.amdsmi = amdsmi
            amdsmi.amdsmi_init()
            handles = amdsmi.amdsmi_get_processor_handles()
            props = torch.cuda.get_device_properties(dev)
            bus = getattr(props, "pci_bus_id", None)
            pick = None
            for h in handles:
                bdf = amdsmi.amdsmi_get_gpu_device_bdf(h)
                if bus is not None and int(bdf.split(":")[1], 16) == int(bus):
                    pick = h
            if pick is None and len(handles) == 1:
                pick = handles[0]
            if pick is None:
                raise RuntimeError("no amdsmi device matches PCI bus %s" % bus)
            self.h = pick
            self.bdf = amdsmi.amdsmi_get_gpu_device_bdf(pick)
        except Exception as e:  # telemetry only: never fail the bench for it
            self.source = "energy unavailable: %r" % (e,)

    def _counter(self):
        r = self.amdsmi.amdsmi_get_energy_count(self.h)
        return r["energy_accumulator"] * r["counter_resolution"] * 1e-6  # uJ -> J

    def _power(self):
        info = self.amdsmi.amdsmi_get_power_info(self.h)
        for key in ("current_socket_power", "socket_power", "average_socket_power"):
            w = info.get(key)
            if isinstance(w, (int, float)) and w > 0:
                return float(w)
        return None

    def _sample(self):
        while not self.stop_ev.is_set():
            try:
                w = self._power()
            except Exception:
                w = None
            self.samples.append((time.perf_counter(), w))
            time.sleep(0.005)

    def start(self):
        self.e0 = None
        if self.h is None:
            return
        try:
            self.e0 = self._counter()
        except Exception:
            self.e0 = None
        self.th.start()

    def stop(self):
        if self.h is None:
            return None
        self.stop_ev.set()
        self.th.join()
        try:
            if self.e0 is not None:
                joules = self._counter() - self.e0
                if joules > 0:
                    self.source = "amdsmi energy counter, device %s" % self.bdf
                    return joules
        except Exception:
            pass
        pts = [(t, w) for t, w in self.samples if w is not None]
        if len(pts) >= 2:
            joules = sum(0.5 * (w0 + w1) * (t1 - t0)
                         for (t0, w0), (t1, w1) in zip(pts, pts[1:]))
            self.source = ("amdsmi socket power sampled every 5 ms (%d samples), device %s; "
                           "the energy counter did not advance" % (len(pts), self.bdf))
            return joules if joules > 0 else None
        self.source = "energy unavailable: counter did not advance, no power samples"
        return None


class MemoryWatch:
    """Peak device memory in use above the level at start(), polled."""

    def __init__(self, torch, dev):
        import threading
        self.torch, self.dev = torch, dev
        self.stop_ev = threading.Event()
        self.min_free = None
        self.th = threading.Thread(target=self._run, daemon=True)

    def _run(self):
        while not self.stop_ev.is_set():
            free, _ = self.torch.cuda.mem_get_info(self.dev)
            self.min_free = free if self.min_free is None else min(self.min_free, free)
            time.sleep(0.002)

    def start(self):
        self.free0, _ = self.torch.cuda.mem_get_info(self.dev)
        self.th.start()

    def stop(self):
        self.stop_ev.set()
        self.th.join()
        return int(self.free0 - self.min_free) if self.min_free is not None else None


# the count kernels' degree bins: middle vertices b by out-degree d+(b)
COUNT_BIN_LIMITS = (32, 256, 2048, 8192)
COUNT_BIN_NAMES = ("d+ <= 32", "d+ 33..256", "d+ 257..2048", "d+ 2049..8192", "d+ > 8192")


def algorithmic_bytes(row_ptr: np.ndarray, col: np.ndarray, chunk: int = 128,
                      bin_limits=COUNT_BIN_LIMITS, stage_grid=None) -> dict:
    """Bytes a count pass must move with no cache reuse.

    B_model_min: the two whole-list schedules (stage the low vertex and stream
    N+(v): 16n + 20m + 4 S_dst; stage the middle vertex and stream N+(u) over
    its in-edges: 16n + 24m + 4 S_src), the smaller of the two.
    bytes: what these kernels' schedule moves -- per middle vertex b with
    d+(b) > 0 and an in-edge chunk: the unit (16 B), its two row pointers (8 B)
    and N+(b) staged once per chunk (4 B each); per in-edge a->b: its packed
    tail range (8 B); per tail element (only x > b can close a triangle): 4 B.
    bytes_by_bin: the same, split by the degree bin of the middle vertex b
    (d+(b) <= 32, <= 256, <= 2048, <= 8192, larger): one entry per bin.
    chunk: in-edges per unit, one for all bins or one per bin.
    stage_grid: per bin, None (N+(b) staged once per unit), or the largest
    grid G of a kernel whose blocks take contiguous stretches of the bin's
    units (in vertex order): with g = min(G, units of the bin) blocks and
    ceil(units / g) units per block, N+(b) is staged once per block that holds
    a unit of b."""
    n = len(row_ptr) - 1
    m = len(col)
    dout = np.diff(row_ptr).astype(np.int64)
    src = np.repeat(np.arange(n, dtype=np.int64), dout)
    row_end = row_ptr[1:].astype(np.int64)[src]
    tail = row_end - np.arange(m, dtype=np.int64) - 1
    live = dout[col] > 0                       # head has out-edges: a unit exists
    probes = int(tail[live].sum())
    in_edges = int(live.sum())
    din = np.bincount(col, minlength=n).astype(np.int64)
    has = (dout > 0) & (din > 0)
    limits = np.asarray(bin_limits, dtype=np.int64)
    nb = len(limits) + 1
    ebin = np.searchsorted(limits, dout[col[live]], side="left")     # bin of each in-edge's b
    vbin = np.searchsorted(limits, dout[has], side="left")           # bin of each middle vertex
    per_bin = np.broadcast_to(np.asarray(chunk, dtype=np.int64), (nb,))
    chunk_v = per_bin[vbin]
    chunks = (din[has] + chunk_v - 1) // chunk_v
    units = int(chunks.sum())
    stagings = chunks.copy()                   # times N+(b) is staged, per vertex
    for bb, grid in enumerate(stage_grid or [None] * nb):
        sel = np.flatnonzero(vbin == bb)         # the bin's vertices, in rank order
        if grid is None or len(sel) == 0:
            continue
        c_b = chunks[sel]
        nu = int(c_b.sum())
        g = min(int(grid), nu)
        per = -(-nu // g)
        end = np.cumsum(c_b)
        first = end - c_b                       # the vertex's units [first, end)
        stagings[sel] = (end - 1) // per - first // per + 1
    staged = int((stagings * dout[has]).sum())
    b = 4 * probes + 8 * in_edges + 4 * staged + 24 * units
    probes_b = np.bincount(ebin, weights=tail[live].astype(np.float64), minlength=nb)
    in_b = np.bincount(ebin, minlength=nb)
    units_b = np.bincount(vbin, weights=chunks.astype(np.float64), minlength=nb)
    staged_b = np.bincount(vbin, weights=(stagings * dout[has]).astype(np.float64), minlength=nb)
    by_bin = [int(4 * round(p_) + 8 * int(i_) + 4 * round(s_) + 24 * round(u_))
              for p_, i_, s_, u_ in zip(probes_b, in_b, staged_b, units_b)]
    # the two whole-list schedules of the survey's model, for context
    s_src = int((dout.astype(np.int64) ** 2).sum())
    s_dst = int(dout[col].sum())
    return {"bytes": b, "bytes_by_bin": by_bin, "probes": probes, "in_edges": in_edges,
            "units": units, "staged": staged, "S_src": s_src, "S_dst": s_dst,
            "B_model_min": min(16 * n + 20 * m + 4 * s_dst, 16 * n + 24 * m + 4 * s_src)}


def count_stage_grid(b: int, strategy: int):
    """Largest grid of bin b's count kernel when its blocks take contiguous
    stretches of units (and stage N+(b) once per stretch), else None: the
    LDS-table strategies 0, 1, 3, 4 with tables of 16 KB or more (launch
    configuration of launch_tc_lds in gc_count.hip: 256 CUs x blocks per CU
    by table size)."""
    if strategy not in (0, 1, 3, 4) or b >= 4:
        return None
    slots = ((1 << (6, 9, 12, 14)[b]) if strategy in (0, 1) else (4 << (4, 7, 10, 12)[b]))
    tbytes = 4 * slots * (2 if strategy in (1, 4) else 1)
    if tbytes < 16384:
        return None
    per_cu = 512 if tbytes <= 16384 else 64 if tbytes <= 32768 else 32 if tbytes <= 65536 else 16
    return 256 * per_cu


def count_kernel_name(b: int, strategy: int) -> str:
    """Kernel that runs degree bin b of the count with a given strategy (the
    strategy numbers of include/gc.h)."""
    if strategy == 2 or b == 4:
        return "gc::k_tc_search"
    if strategy == 5:
        return "gc::k_tc_group<6, 16>" if b == 0 else "gc::k_tc_group<9, 64>"
    if strategy in (0, 1):
        return "gc::k_tc_lds<gc::LinTable<%d> >" % ((6, 9, 12, 14)[b] + strategy)
    return "gc::k_tc_lds<gc::BucketTable<%d> >" % ((4, 7, 10, 12)[b] + (strategy == 4))


def profiled_traffic(kernel: str, workload: str, scale: int, ef: int, seed: int, strategy,
                     tile=None):
    """HBM bytes of one launch of `kernel` from the committed rocprofv3
    counter summary (FETCH_SIZE + WRITE_SIZE, each scaled by a plain
    elementwise kernel of known size), if that summary was taken on this
    workload with these strategies and tiles and the count kernels' current source;
    else None (the kernel changed since the counters were taken)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "tc_count_rmat_s24.md")
    src = os.path.join(ROOT, "paper_1708_06866_amd", "csrc", "gc_count.hip")
    if not (os.path.exists(path) and os.path.exists(src)) or strategy is None:
        return None
    kv, traffic = {}, {}
    for line in open(path):
        if line.startswith("traffic_bytes_per_launch "):
            name, val = line[len("traffic_bytes_per_launch "):].rsplit("=", 1)
            traffic[name.strip()] = int(val)
        elif ":" in line and not line.startswith(("#", "|", " ")):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    try:
        ok = (kv["count_source_sha256"] == hashlib.sha256(open(src, "rb").read()).hexdigest()
              and kv["workload"] == "%s %d %d %d" % (workload, scale, ef, seed)
              and [int(x) for x in kv["strategy"].split()] == list(strategy)
              and [int(x) for x in kv.get("tile", "128 128 128 128 128").split()]
              == list(tile or [128] * 5))
        return traffic.get(kernel) if ok else None
    except (KeyError, ValueError):
        return None


def host_cpu() -> dict:
    """The host's CPU model (/proc/cpuinfo) and the cores this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "cores_available": len(os.sched_getaffinity(0)),
            "os_cpu_count": os.cpu_count()}


def cpu_baseline(scale: int, ef: int, seed: int, all_cores_scale: int) -> dict:
    """The oracle as it stands, timed on the host's cores, as context.

    value: one thread (the paper's serial mode) on R-MAT of `scale`, a bounded
    sample of the benchmark's family: normalise + triangle count + truss
    decomposition.  all_cores: the triangle count on R-MAT of
    `all_cores_scale` with its outer loop dealt over every core this process
    may use (per-thread int64 partials; the count equals the serial one),
    after a serial normalisation."""
    import graphgen as gg
    import oracle
    src, dst, n = gg.rmat(scale, ef, seed=seed)
    t0 = time.perf_counter()
    u, v = oracle.normalise(src, dst, n)
    oracle.triangle_count(n, u, v)
    oracle.truss_decomposition(n, u, v, "search")
    dt = time.perf_counter() - t0
    out = {"value": len(u) / dt, "unit": "edges/s", "cores": 1, "kind": "oracle",
           "sample": "R-MAT scale %d ef %d seed %d (m=%d): normalise + triangle count + "
                     "truss decomposition, %.1f s single-threaded" % (scale, ef, seed, len(u), dt),
           "seconds": round(dt, 2), "host": host_cpu()}
    del src, dst, u, v
    if all_cores_scale > 0:
        threads = out["host"]["cores_available"]
        src, dst, n = gg.rmat(all_cores_scale, ef, seed=seed)
        t0 = time.perf_counter()
        u, v = oracle.normalise(src, dst, n)
        t1 = time.perf_counter()
        T = oracle.triangle_count_threads(n, u, v, threads)
        t2 = time.perf_counter()
        out["all_cores"] = {
            "threads": threads, "workload": "R-MAT scale %d ef %d seed %d" % (
                all_cores_scale, ef, seed),
            "m": int(len(u)), "triangles": T, "normalise_s": round(t1 - t0, 2),
            "count_s": round(t2 - t1, 2), "count_edges_per_s": len(u) / (t2 - t1),
            "edges_per_s": len(u) / (t2 - t0),
            "what": "serial normalisation, then the triangle count over %d threads "
                    "(its adjacency build is serial)" % threads}
    return out


def batch_workload(n_graphs: int, seed: int = 1000, max_scale: int = 16):
    """C4-style mix: half R-MAT (scale uniform 8..max_scale, i.e. vertex
    counts log-uniform; edge factor uniform 8..32), half random geometric
    graphs on the torus (n = 2^10..2^14 log-uniform, mean degree 20), shuffled;
    graph i uses seed + i."""
    import graphgen as gg
    rng = np.random.default_rng(seed)
    kinds = np.array([0] * (n_graphs // 2) + [1] * (n_graphs - n_graphs // 2))
    rng.shuffle(kinds)
    graphs = []
    for i, kd in enumerate(kinds):
        if kd == 0:
            sc = int(rng.integers(8, max_scale + 1))
            ef = int(rng.integers(8, 33))
            graphs.append(gg.rmat(sc, ef, seed=seed + i))
        else:
            n = 1 << int(rng.integers(10, 15))
            graphs.append(gg.rgg(n, 20.0, seed=seed + i))
    return graphs


def stream_bandwidth(torch, dev, gib: int = 4) -> dict:
    """Achievable HBM bandwidth on this GPU, for the roofline beside the
    published peak: a device copy of `gib` GiB (read + write), best of 5,
    timed with HIP events."""
    n = (gib << 30) // 4
    x = torch.ones(n, dtype=torch.int32, device=dev)
    y = torch.empty_like(x)

    def best(fn):
        t = []
        for _ in range(6):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            b.synchronize()
            t.append(a.elapsed_time(b) / 1000.0)
        return min(t[1:])
    c = best(lambda: y.copy_(x))
    del x, y
    torch.cuda.empty_cache()
    return {"copy_GBps": 2 * n * 4 / c / 1e9, "bytes": n * 4}


def bench_batch(gc, torch, dev, n_graphs: int, max_scale: int) -> dict:
    """Batched path vs one graph per call on the same GPU, exact agreement:
    per-graph triangle count + 4-truss edge count.  batched_s: build the
    batch, count, 4-truss (recording both launch sequences); replay_s: count
    and 4-truss again on the built batch (replays of the recorded
    sequences)."""
    t = time.perf_counter()
    graphs = batch_workload(n_graphs, max_scale=max_scale)
    log("batch: generated %d graphs in %.1fs" % (len(graphs), time.perf_counter() - t))
    srcs = [torch.from_numpy(g[0]) for g in graphs]
    dsts = [torch.from_numpy(g[1]) for g in graphs]
    off = np.zeros(len(graphs) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(g[0]) for g in graphs])
    nv = [g[2] for g in graphs]
    d_src = torch.cat(srcs).to(dev)
    d_dst = torch.cat(dsts).to(dev)
    per_src = [x.to(dev) for x in srcs]
    per_dst = [x.to(dev) for x in dsts]
    torch.cuda.synchronize()

    def run_batch():
        b = gc.gc_batch_build(d_src, d_dst, off, nv)
        T = b.triangle_count()
        _, mk = b.ktruss(4)
        torch.cuda.synchronize()
        return b, T.cpu().numpy(), mk.cpu().numpy()

    b, _, _ = run_batch()          # warm up (code objects, allocator)
    st, _ = b.autotune()
    b.free()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b, T_b, mk_b = run_batch()
    t_batch = time.perf_counter() - t0
    edges_total = int(b.edge_offsets[-1])
    # the same batch again: both halves replay their recorded launch
    # sequences (count, and the 4-truss levels)
    replay = []
    for _ in range(3):
        t0 = time.perf_counter()
        T_r = b.triangle_count()
        _, mk_r = b.ktruss(4)
        torch.cuda.synchronize()
        replay.append(time.perf_counter() - t0)
        assert np.array_equal(T_r.cpu().numpy(), T_b) and np.array_equal(mk_r.cpu().numpy(), mk_b)
    b.free()

    # one graph per call, same GPU, same stream
    T_c = np.zeros(len(graphs), np.int64)
    mk_c = np.zeros(len(graphs), np.int64)
    for i in range(min(8, len(graphs))):   # warm up
        g = gc.gc_build_csr(per_src[i], per_dst[i], nv[i])
        g.triangle_count()
        g.free()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(len(graphs)):
        g = gc.gc_build_csr(per_src[i], per_dst[i], nv[i])
        T_c[i] = g.triangle_count()
        mk_c[i] = g.ktruss(4)[1]
        g.free()
    torch.cuda.synchronize()
    t_call = time.perf_counter() - t0
    assert np.array_equal(T_b, T_c) and np.array_equal(mk_b, mk_c), "batched != per-call"
    return {"graphs": len(graphs), "edges": edges_total, "raw_pairs": int(off[-1]),
            "batched_s": round(t_batch, 4), "per_call_s": round(t_call, 4),
            "replay_s": round(float(np.median(replay)), 4),
            "replay_edges_per_s": edges_total / float(np.median(replay)),
            "batched_edges_per_s": edges_total / t_batch, "per_call_edges_per_s": edges_total / t_call,
            "speedup": t_call / t_batch, "autotuned_strategy": st.tolist(),
            "exact_agreement": True,
            "workload": "half R-MAT (scale 8..%d, ef 8..32), half torus RGG (n 2^10..2^14, "
                        "degree 20); per graph: triangle count + 4-truss" % max_scale}


def serve_pool(n_graphs: int, seed: int = 5000, big_max: int = 18):
    """Serving pool: R-MAT ef 16, scale uniform 10..14 with p = 0.9, else
    uniform 15..big_max."""
    import graphgen as gg
    rng = np.random.default_rng(seed)
    out = []
    for j in range(n_graphs):
        sc = int(rng.integers(10, 15)) if rng.random() < 0.9 else int(rng.integers(15, big_max + 1))
        out.append(gg.rmat(sc, 16, seed=seed + j))
    return out


def bench_serve(gc, n_graphs: int, n_requests: int, big_max: int, budget: int) -> dict:
    """Serving at a fixed offered load: Poisson arrivals at 0.7 x the
    one-request-at-a-time capacity, half triangle counts, half 4-truss sizes,
    on a pool of R-MAT graphs (scale 10..14 with p = 0.9, else 15..big_max).
    Every run starts from a fresh server with an empty device cache, so
    first touches (builds) happen inside the trace, and the HBM budget is
    below the pool's resident footprint, so graphs are evicted and rebuilt.
    The same trace is served one request at a time (per call) and with
    continuous batching; every answer must agree."""
    import threading
    t = time.perf_counter()
    pool = serve_pool(n_graphs, big_max=big_max)
    log("serve: generated %d graphs (%d pairs) in %.1fs" % (
        len(pool), sum(len(g[0]) for g in pool), time.perf_counter() - t))
    rng = np.random.default_rng(7)
    reqs = [(int(rng.integers(0, n_graphs)), int(rng.random() < 0.5)) for _ in range(n_requests)]

    def make_server(mode):
        srv = gc.Server(budget, mode=mode)
        for s_, d_, n_ in pool:
            srv.add_graph(s_, d_, n_)
        return srv

    def run(mode, trace_gaps, count):
        srv = make_server(mode)
        trace = reqs[:count]
        tickets = [None] * len(trace)

        def submitter():
            t_next = time.monotonic()
            for i, (g, kind) in enumerate(trace):
                if trace_gaps is not None:
                    t_next += trace_gaps[i]
                    dt = t_next - time.monotonic()
                    if dt > 0:
                        time.sleep(dt)
                tickets[i] = srv.submit(g, kind, 4 if kind else 0)
        th = threading.Thread(target=submitter)
        t0 = time.monotonic()
        th.start()
        th.join()
        res = [srv.wait(tk) for tk in tickets]
        wall = time.monotonic() - t0
        stats = srv.stats()
        srv.close()
        # latency percentiles over the requests after a warm-up tenth
        lat = np.array([r["t_done"] - r["t_submit"] for r in res[len(res) // 10:]])
        edges = sum(r["edges"] for r in res)
        log("serve: mode %d %s: %.1f s, %s" % (mode, "Poisson" if trace_gaps is not None
                                                else "saturated", wall, stats))
        return res, wall, lat, edges, stats

    # capacity of the one-at-a-time path: the first quarter of the trace
    # submitted at once (a cold cache, as the timed runs start)
    n_sat = max(1, len(reqs) // 4)
    res_sat1, wall_sat1, _, edges_sat, _ = run(1, None, n_sat)
    cap = n_sat / wall_sat1
    lam = 0.7 * cap
    gaps = np.random.default_rng(8).exponential(1.0 / lam, len(reqs))
    res_p1, wall_p1, lat_p1, edges, stats1 = run(1, gaps, len(reqs))
    res_p0, wall_p0, lat_p0, _, stats0 = run(0, gaps, len(reqs))
    res_sat0, wall_sat0, _, _, _ = run(0, None, n_sat)
    vals = [r["value"] for r in res_p1]
    assert [r["value"] for r in res_p0] == vals, "results differ between modes"
    assert [r["value"] for r in res_sat1] == vals[:n_sat] == [r["value"] for r in res_sat0]
    assert all(r["status"] == 0 for r in res_sat1 + res_p1 + res_sat0 + res_p0)
    pct = lambda a, q: float(np.percentile(a, q) * 1000.0)
    keep = ("builds", "evictions", "peak_bytes_charged", "deferred")
    return {
        "requests": len(reqs), "graphs": n_graphs, "offered_load_req_per_s": lam,
        "budget_bytes": budget,
        "per_call": {"p50_ms": pct(lat_p1, 50), "p99_ms": pct(lat_p1, 99),
                     "edges_per_s_at_load": edges / wall_p1,
                     "saturated_edges_per_s": edges_sat / wall_sat1,
                     "saturated_req_per_s": n_sat / wall_sat1,
                     **{k: stats1[k] for k in keep}},
        "continuous_batching": {"p50_ms": pct(lat_p0, 50), "p99_ms": pct(lat_p0, 99),
                                "edges_per_s_at_load": edges / wall_p0,
                                "saturated_edges_per_s": edges_sat / wall_sat0,
                                "saturated_req_per_s": n_sat / wall_sat0,
                                "max_batch": stats0["max_batch"], "batches": stats0["batches"],
                                "truss_batches": stats0["truss_batches"],
                                "max_truss_batch": stats0["max_truss_batch"],
                                **{k: stats0[k] for k in keep}},
        "exact_agreement": True,
        "workload": "R-MAT ef 16 pool, scale 10..14 (p=0.9) / 15..%d; 50%% triangle count, "
                    "50%% 4-truss size; Poisson arrivals at 0.7 x per-call capacity (saturated "
                    "rates over the first quarter of the trace submitted at once); every run "
                    "from an empty device cache (first touches inside the trace) under a "
                    "%.0f GiB budget; latency percentiles over the requests after the first "
                    "tenth" % (big_max, budget / (1 << 30)),
    }


def bench_contrast(gc, torch, dev, scale: int, ef: int, seed: int, steps: int) -> dict:
    """The paired contrast of the full-size workload: an Erdos-Renyi G(n, M)
    graph with n = 2^scale and M = ef * n pairs (mean degree about 2 ef, low
    clustering), the same step (build + count + full decomposition), after
    autotuning the count on it and one untimed step."""
    import graphgen as gg
    t = time.perf_counter()
    n = 1 << scale
    src, dst = gg.er(n, ef * n, seed=seed)[:2]
    log("contrast: generated %d ER pairs in %.1fs" % (len(src), time.perf_counter() - t))
    d_src = torch.from_numpy(src).to(dev)
    d_dst = torch.from_numpy(dst).to(dev)
    del src, dst
    g = gc.gc_build_csr(d_src, d_dst, n)
    strategy, _ = g.autotune()
    g.free()
    stream = torch.cuda.current_stream()
    tau = None
    rows = []
    for i in range(steps + 1):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record(stream)
        g = gc.gc_build_csr(d_src, d_dst, n)
        ev[1].record(stream)
        T = g.triangle_count()
        ev[2].record(stream)
        if tau is None:
            tau = torch.empty(max(g.m, 1), dtype=torch.int32, device=dev)
        _, kmax = g.truss_decomposition(out=tau)
        ev[3].record(stream)
        torch.cuda.synchronize()
        m = g.m
        bins = g.count_times()
        g.free()
        if i > 0:
            rows.append([ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2]),
                         ev[2].elapsed_time(ev[3]), ev[0].elapsed_time(ev[3])] + list(bins))
    r = np.mean(np.array(rows), axis=0)
    return {"workload": "Erdos-Renyi G(n, M), n = 2^%d, M = %d n pairs, seed %d; step = build "
                        "CSR + triangle count + full truss decomposition" % (scale, ef, seed),
            "m_edges": int(m), "triangles": int(T), "kmax": int(kmax),
            "edges_per_s": m / (r[3] / 1000.0), "ms_per_step": float(r[3]),
            "phases_ms": {"build": float(r[0]), "triangle_count": float(r[1]),
                          "decomposition": float(r[2])},
            "count_ms_by_bin": [float(x) for x in r[4:]],
            "autotuned_strategy": strategy.tolist(), "steps": steps}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat", choices=["rmat", "er"])
    ap.add_argument("--scale", type=int, default=24)
    ap.add_argument("--ef", type=int, default=16)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--input", default=None,
                    help="edge file (TSV triples or Matrix Market) instead of a generated graph; "
                         "read on the host before timing")
    ap.add_argument("--cpu-scale", type=int, default=18)
    ap.add_argument("--cpu-all-cores-scale", type=int, default=20,
                    help="R-MAT scale of the all-cores oracle count (0 = skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-decomposition", action="store_true",
                    help="step = build + count only")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the per-bin strategy autotuner (run before the timed steps)")
    ap.add_argument("--contrast-steps", type=int, default=2,
                    help="timed steps of the Erdos-Renyi contrast of the same size (0 = skip)")
    ap.add_argument("--batch-graphs", type=int, default=4096,
                    help="graphs in the batched-path comparison (0: skip)")
    ap.add_argument("--batch-max-scale", type=int, default=16)
    ap.add_argument("--serve-requests", type=int, default=20000,
                    help="requests in the serving comparison (0: skip)")
    ap.add_argument("--serve-graphs", type=int, default=1024)
    ap.add_argument("--serve-big-max", type=int, default=22)
    ap.add_argument("--serve-budget-gib", type=float, default=64.0,
                    help="HBM budget of the server (below the pool's resident footprint)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run one elementwise int32 kernel over 1 GiB (reads 1 GiB, "
                         "writes 1 GiB) so HBM counters can be scaled against known bytes")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: multi-GPU execution (sharding work units "
              "by byte weight, exchanging support deltas) is designed but not implemented",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1708_06866_amd as gc
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.copy_calibration:
        x = torch.ones(1 << 28, dtype=torch.int32, device=dev)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        torch.neg(x, out=y)
        torch.cuda.synchronize()
        log("copy calibration: elementwise kernel read %d B, wrote %d B" % (x.numel() * 4, y.numel() * 4))
        del x, y

    t = time.perf_counter()
    if args.input:
        src, dst, n = gc.gc_read_edges(args.input)
        log("read %d pairs from %s in %.1fs" % (len(src), args.input, time.perf_counter() - t))
    else:
        src, dst, n = gen_inputs(args.workload, args.scale, args.ef, args.seed)
        log("generated %d pairs in %.1fs" % (len(src), time.perf_counter() - t))
    read_s = time.perf_counter() - t
    d_src = torch.from_numpy(src).to(dev)
    d_dst = torch.from_numpy(dst).to(dev)
    del src, dst
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    tau_buf = None
    record_stats = {}
    count_ms_steps = []   # per step: kernel ms of each degree bin's count launch

    tuned = None
    if not args.no_autotune:
        # the autotuner times every count strategy per degree bin on this graph
        # and writes its choice to a cache file that later builds read
        import tempfile
        os.environ.setdefault("GC_AUTOTUNE_CACHE",
                              os.path.join(tempfile.gettempdir(), "gc_autotune_%d.txt" % os.getpid()))
        g = gc.gc_build_csr(d_src, d_dst, n)
        st, ms = g.autotune()
        tile = g.count_config()[1]
        g.free()
        tuned = {"strategy": st.tolist(), "tile": tile.tolist(),
                 "ms": [[round(float(x), 3) for x in row] for row in ms]}
        log("autotune: strategy per bin %s, tile per bin %s; ms per bin x strategy (at the tile) %s"
            % (tuned["strategy"], tuned["tile"], tuned["ms"]))

    def step(record):
        nonlocal tau_buf
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record(stream)
        g = gc.gc_build_csr(d_src, d_dst, n)
        ev[1].record(stream)
        T = g.triangle_count()
        ev[2].record(stream)
        count_ms_steps.append(g.count_times())
        kmax = None
        if not args.no_decomposition:
            if tau_buf is None or tau_buf.numel() < g.m:
                tau_buf = torch.empty(max(g.m, 1), dtype=torch.int32, device=dev)
            _, kmax = g.truss_decomposition(out=tau_buf)
        ev[3].record(stream)
        if kmax is not None:
            record_stats.update(g.truss_stats())
        m = g.m
        record.append((ev, T, kmax, m))
        return g

    # warmup
    recs = []
    for i in range(args.warmup):
        g = step(recs)
        g.free()
        log("warmup step %d done" % i)
    torch.cuda.synchronize()

    # algorithmic bytes of the count pass (host-side, outside the timed region)
    g = gc.gc_build_csr(d_src, d_dst, n)
    _, row_ptr, col, _ = g.oriented()
    st_used = tuned["strategy"] if tuned else [0, 0, 0, 0, 2]
    ab = algorithmic_bytes(row_ptr.cpu().numpy(), col.cpu().numpy(),
                           chunk=tuned["tile"] if tuned else 128,
                           stage_grid=[count_stage_grid(b, st_used[b]) for b in range(5)])
    g.free()
    del row_ptr, col
    torch.cuda.synchronize()

    recs = []
    count_ms_steps.clear()
    torch.cuda.synchronize()
    energy = EnergyMeter(torch, dev)
    memory = MemoryWatch(torch, dev)
    graph_bytes = 0
    energy.start()
    memory.start()
    t0 = time.perf_counter()
    for i in range(args.steps):
        g = step(recs)
        if i == 0:
            graph_bytes = g.info()[2]
        g.free()
        log("step %d done" % i)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    joules = energy.stop()
    peak_bytes = memory.stop()

    m = recs[-1][3]
    T = recs[-1][1]
    kmax = recs[-1][2]
    build_steps = [r[0][0].elapsed_time(r[0][1]) for r in recs]
    tc_steps = [r[0][1].elapsed_time(r[0][2]) for r in recs]
    dec_steps = [r[0][2].elapsed_time(r[0][3]) for r in recs]
    build_ms = np.mean(build_steps)
    tc_ms = np.mean(tc_steps)
    dec_ms = np.mean(dec_steps)
    ms_per_step = wall * 1000.0 / args.steps
    value = m / (ms_per_step / 1000.0)

    # The count pass against the HBM roofline.  Its dominant kernel (the
    # launch of the degree bin that takes longest) is measured on its own
    # algorithmic bytes: the schedule's tail model (4 B per tail element
    # streamed, 8 B per in-edge, 4 B per staged element each time N+(b) is
    # staged -- once per unit, or once per block stretch where the kernel's
    # blocks take contiguous stretches of units -- and 24 B per unit) over
    # the bin's kernel time from HIP events around that launch on
    # the stream it runs on, averaged over the timed steps.  The whole pass is
    # given beside it, and so is B_TC = min(16n + 20m + 4 S_dst, 16n + 24m +
    # 4 S_src), the whole-list model of Alg. 3 (every element of the streamed
    # lists read per unit): the kernels stream only the tails, so B_TC
    # overstates the bytes they move.
    bin_ms = np.mean(np.array(count_ms_steps, dtype=np.float64), axis=0)
    dom = int(np.argmax(bin_ms))
    strategy = tuned["strategy"] if tuned else None
    dom_kernel = count_kernel_name(dom, strategy[dom] if strategy else (2 if dom == 4 else 0))
    dom_bytes = ab["bytes_by_bin"][dom]
    achieved = dom_bytes / (bin_ms[dom] / 1000.0) / 1e9
    pass_ms = float(bin_ms.sum())
    bw = stream_bandwidth(torch, dev)
    log("achievable bandwidth: copy %.0f GB/s (read + write)" % bw["copy_GBps"])
    traffic = None if args.input else profiled_traffic(
        dom_kernel, args.workload, args.scale, args.ef, args.seed, strategy,
        tuned["tile"] if tuned else None)
    out = {
        "metric": "triangle-count and k-truss edges/sec at R-MAT scale 24",
        "value": value,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "file" if args.input else "synthetic",
        "config": {
            "workload": "%s; step = build CSR from raw pairs in HBM + triangle count + %s" % (
                ("edge file %s" % os.path.basename(args.input)) if args.input else
                "%s scale %d edge factor %d seed %d%s" % (
                    "R-MAT (0.57,0.19,0.19,0.05)" if args.workload == "rmat" else "ER G(n,M)",
                    args.scale, args.ef, args.seed,
                    ", vertex ids permuted" if args.workload == "rmat" else ""),
                "count only" if args.no_decomposition else "full truss decomposition"),
            "n_vertices": int(n), "m_edges": int(m), "adjacency_entries": int(2 * m),
            "triangles": int(T), "kmax": kmax,
        },
        "phases_ms": {"build": build_ms, "triangle_count": tc_ms, "decomposition": dec_ms},
        # every timed step's phases (HIP events on the step's stream), for the spread
        "phases_ms_per_step": {"build": build_steps, "triangle_count": tc_steps,
                               "decomposition": dec_steps},
        "autotune": tuned,
        "decomposition_stats": record_stats or None,
        # the decomposition's dominant kernel (k_peel) is bound by the L1
        # misses a CU keeps in flight, not by HBM bandwidth: its rate is
        # given in candidate third vertices examined per second of the
        # decomposition phase
        "peel_candidates_per_s": (record_stats["candidates"] / (dec_ms / 1000.0)
                                  if record_stats and dec_ms > 0 else None),
        # the decomposition's bytes by a per-candidate model: each candidate
        # reads its list entry (4 B) and its edge's state (1 B); each search
        # ends on one 4-byte key; each destroyed triangle updates two
        # supports (4-byte read-modify-write each); over the phase time
        "peel_model": (lambda mb: {
            "model_bytes": mb, "GBps": mb / (dec_ms / 1000.0) / 1e9,
            "frac": mb / (dec_ms / 1000.0) / 1e9 / HBM_PEAK_GBS,
            "model": "5 B per candidate + 4 B per search + 16 B per destroyed triangle",
            "note": "the peel is bound by the L1 misses a CU keeps in flight (binary "
                    "searches), not by these bytes"})(
            5 * record_stats["candidates"] + 4 * record_stats["searches"]
            + 16 * record_stats["triangles_destroyed"]) if record_stats and dec_ms > 0 else None,
        "tc_edges_per_s": m / (tc_ms / 1000.0),
        # Sec. IV metrics beside the rate: energy of the timed steps from the
        # GPU's energy counter, rate per watt, and device memory
        "energy": ({"joules_per_step": joules / args.steps, "avg_watts": joules / wall,
                    "edges_per_s_per_watt": value / (joules / wall),
                    "source": energy.source} if joules
                   else {"error": energy.source}),
        "memory": {"graph_handle_bytes": int(graph_bytes),
                   "step_peak_device_bytes": peak_bytes,
                   "source": "hipMemGetInfo polled every 2 ms during the timed steps; "
                             "graph handle from gc_graph_info"},
        "input_read_s": read_s,
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": "%s: triangle count, degree bin %d (%s)" % (
                dom_kernel, dom, COUNT_BIN_NAMES[dom]),
            "kernel_ms": float(bin_ms[dom]),
            "algorithmic_bytes": dom_bytes,
            "algorithmic_model": "per launch: 4 B per tail element streamed + 8 B per in-edge "
                                 "+ 4 B per staged element each time N+(b) is staged (once per "
                                 "block stretch of the bin's units for the large-table kernels, "
                                 "else once per unit) + 24 B per unit, over the bin's units",
            "traffic_source": "profiles/tc_count_rmat_s24.md (rocprofv3 FETCH_SIZE + WRITE_SIZE "
                              "per launch, calibrated on an elementwise kernel; null unless "
                              "taken on the current count source with these strategies)",
            "count_ms_by_bin": [float(x) for x in bin_ms],
            "tail_model_bytes_by_bin": ab["bytes_by_bin"],
            "pass": {"kernel_ms": pass_ms, "tail_model_bytes": ab["bytes"],
                     "achieved": ab["bytes"] / (pass_ms / 1000.0) / 1e9,
                     "frac": ab["bytes"] / (pass_ms / 1000.0) / 1e9 / HBM_PEAK_GBS,
                     "B_TC": ab["B_model_min"], "S_src": ab["S_src"], "S_dst": ab["S_dst"],
                     "B_TC_per_s_GBps": ab["B_model_min"] / (pass_ms / 1000.0) / 1e9,
                     "B_TC_note": "whole-list model of Alg. 3, context only: the kernels "
                                  "stream only list tails, so B_TC / t overstates moved bytes",
                     "probes": ab["probes"]},
            "achievable_copy_GBps": bw["copy_GBps"],
            "frac_of_achievable_copy": achieved / bw["copy_GBps"],
        },
    }
    del d_src, d_dst
    torch.cuda.empty_cache()
    if args.contrast_steps > 0 and not args.input and args.workload == "rmat":
        log("contrast: Erdos-Renyi n = 2^%d ..." % args.scale)
        out["er_contrast"] = bench_contrast(gc, torch, dev, args.scale, args.ef, 2,
                                            args.contrast_steps)
        log("contrast: %s" % json.dumps(out["er_contrast"]))
    if args.batch_graphs > 0:
        log("batched path: %d graphs ..." % args.batch_graphs)
        out["batch"] = bench_batch(gc, torch, dev, args.batch_graphs, args.batch_max_scale)
        log("batch: %s" % json.dumps(out["batch"]))
    if args.serve_requests > 0:
        log("serving: %d requests on %d graphs ..." % (args.serve_requests, args.serve_graphs))
        out["serve"] = bench_serve(gc, args.serve_graphs, args.serve_requests,
                                   args.serve_big_max, int(args.serve_budget_gib * (1 << 30)))
        log("serve: %s" % json.dumps(out["serve"]))
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on R-MAT scale %d ..." % args.cpu_scale)
        out["cpu_baseline"] = cpu_baseline(args.cpu_scale, args.ef, args.seed,
                                           args.cpu_all_cores_scale)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
