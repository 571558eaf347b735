"""Benchmark: dense-tableau simplex pivots on one MI355X.

Default workload: one dense LP, m = n = 8192, FP64, generator seed 0 (A
integer uniform [1,100], b uniform [1000 s, 10000 s] with s = n/64, c integer
uniform [1,100]).  One step = one lp_solve_dense_ex call through the C ABI:
Table 1 build, the whole pivot loop on the device (pricing, ratio test,
pivot-row division, rank-1 update of the (m+1) x (n+m+1) tableau) and the
solution read-out.  Inputs are resident in HBM before the timed region.

Prints one JSON line (rank 0).  `value` is pivots per second over the K timed
steps; `roofline` relates the persistent kernel's algorithmic bytes
(16 (m+1)(n+m+1) per pivot) to its average duration measured with HIP events
on the stream the kernel runs on, and gives the measured HBM traffic rate
from the committed rocprofv3 counters; `cpu_baseline` times the CPU oracle
on a bounded sample of the same LP (its first pivots) on this host, with all
the cores the process may use and with one thread.  The same line carries
the rest of the metric: the same LP on the other schedules, the 64 x 64 LP
(`small_lp`), the shape sweep (`shapes`), the batched workload (`batch`) and
the served workload at three arrival rates (`serve`).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "pivots/s + HBM GB/s (8192x8192 FP64); batched LPs/s; p50/p99 served latency"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_cpu():
    """CPU model, sockets and physical cores of this host (from
    /proc/cpuinfo), and the logical CPUs this process may run on."""
    model, phys, cores_per = "unknown", set(), {}
    try:
        with open("/proc/cpuinfo") as f:
            cur = {}
            for line in f.read().splitlines() + [""]:
                if not line.strip():
                    if cur:
                        model = cur.get("model name", model)
                        pid = cur.get("physical id", "0")
                        phys.add(pid)
                        cores_per[pid] = int(cur.get("cpu cores", "1"))
                    cur = {}
                    continue
                k, _, v = line.partition(":")
                cur[k.strip()] = v.strip()
    except OSError:
        pass
    sockets = max(len(phys), 1)
    physical = sum(cores_per.values()) if cores_per else (os.cpu_count() or 1)
    allowed = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return {"model": model, "sockets": sockets, "physical_cores": physical, "logical_cpus_allowed": allowed}


def _oracle_rate(A, b, c, target_s: float, samples: int, lib_path=None):
    """Oracle pivots/s on the first pivots of (A, b, c): each sample runs the
    oracle with max_iter = 0 (Table 1 build only) and with max_iter = K; the
    difference over K is the time per pivot.  K is sized so that the pivot
    part of a sample takes about target_s / samples.  Returns the median rate
    and the samples."""
    import numpy as np

    import oracle

    def timed(k):
        t0 = time.perf_counter()
        r = oracle.solve(A, b, c, max_iter=k, lib_path=lib_path)
        return time.perf_counter() - t0, r.iterations

    t_build, _ = timed(0)
    t2, it2 = timed(2)
    per = max((t2 - t_build) / max(it2, 1), 1e-9)
    K = int(max(2, min(10_000, target_s / samples / per)))
    rates, Ks = [], []
    for _ in range(samples):
        tb, _ = timed(0)
        tk, it = timed(K)
        rates.append(max(it, 1) / max(tk - tb, 1e-9))
        Ks.append(it)
    return float(np.median(rates)), rates, Ks[0]


def host_triad_gbps(threads: int, mib: int = 1024, reps: int = 5):
    """STREAM-triad bandwidth of this host, a = b + s c on three float64
    arrays of `mib` MiB each with `threads` CPU threads (torch's CPU kernels),
    counted as 3 x the array bytes per pass; best of `reps`."""
    import torch
    prev = torch.get_num_threads()
    torch.set_num_threads(threads)
    try:
        n = mib * (1 << 20) // 8
        b = torch.ones(n, dtype=torch.float64)
        c = torch.full((n,), 2.0, dtype=torch.float64)
        a = torch.empty(n, dtype=torch.float64)
        best = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            torch.add(b, c, alpha=3.0, out=a)
            best = min(best, time.perf_counter() - t0)
        return 3 * n * 8 / best / 1e9
    finally:
        torch.set_num_threads(prev)


def cpu_baseline(m: int, n: int, seed: int, generator: str, target_s: float, samples: int = 3):
    """The CPU oracle on this host (a reported baseline, never the target),
    timed in a child process that touches no GPU, with the OpenMP threads
    pinned to cores (OMP_PROC_BIND=close, OMP_PLACES=cores unless set): the
    OpenMP runtime reads those when it starts, and in this process it
    started with torch."""
    import subprocess
    env = dict(os.environ)
    env.setdefault("OMP_PROC_BIND", "close")
    env.setdefault("OMP_PLACES", "cores")
    # The host as this (unpinned) process sees it: the child's OpenMP runtime
    # binds its initial thread to one core as it starts.
    spec = json.dumps({"m": m, "n": n, "seed": seed, "generator": generator, "target_s": target_s,
                       "samples": samples, "host": host_cpu()})
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-child", spec], env=env,
                       capture_output=True, text=True, timeout=max(300.0, 4 * target_s))
    if r.returncode != 0:
        raise RuntimeError(f"CPU baseline child failed ({r.returncode}): {r.stderr[-2000:]}")
    out = json.loads(r.stdout.strip().splitlines()[-1])
    out["pinning"] = f"OMP_PROC_BIND={env['OMP_PROC_BIND']} OMP_PLACES={env['OMP_PLACES']}"
    return out


def _cpu_baseline_child(spec: str):
    """Body of cpu_baseline in its child: the same LP from the generator, the
    oracle with every physical core this process may use (the OpenMP build of
    the same source: Step 5's rows in threads, every value unchanged) and with
    one thread, median of `samples` samples each; one JSON line."""
    q = json.loads(spec)
    # torch first: the oracle's OpenMP build then shares torch's OpenMP
    # runtime (pinned from this process's environment) instead of starting a
    # second one whose idle threads would spin beside torch's during the
    # triad.
    import torch  # noqa: F401
    from paper_1804_04737_amd import lpgen
    gen = lpgen.paper_lp if q["generator"] == "paper" else lpgen.dense_lp
    A, b, c = gen(q["m"], q["n"], q["seed"])
    print(json.dumps(_cpu_baseline_here(A, b, c, q["target_s"], q["samples"], q["host"])), flush=True)


def _cpu_baseline_here(A, b, c, target_s: float, samples: int, host: dict):
    import oracle
    omp_env = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    threads = min(host["physical_cores"], host["logical_cpus_allowed"])
    if omp_env > 0:
        threads = min(threads, omp_env)
    lib = oracle.load_omp()
    used = lib.oracle_threads(threads)
    multi, multi_s, k_multi = _oracle_rate(A, b, c, target_s * 0.5, samples, lib_path=oracle._LIB_OMP)
    single, single_s, k_single = _oracle_rate(A, b, c, target_s * 0.5, samples)
    m, n = A.shape
    # The oracle on its own roofline: its Step 5 streams the tableau like the
    # GPU's sweep, 16 (m+1)(n+m+1) bytes per pivot.
    bpp = 16.0 * (m + 1) * (n + m + 1)
    triad_multi, triad_single = host_triad_gbps(used), host_triad_gbps(1)
    host.update({"stream_triad_GBps": round(triad_multi, 1), "stream_triad_GBps_one_thread": round(triad_single, 1)})
    return {"value": multi, "unit": "pivots/s", "cores": used, "kind": "oracle",
            "effective_GBps": round(multi * bpp / 1e9, 1),
            "frac_of_host_triad": round(multi * bpp / 1e9 / triad_multi, 3),
            "sample": f"first {k_multi} pivots of the same {m}x{n} LP per sample, median of {samples} samples "
                      f"(each: oracle run with max_iter=K minus a max_iter=0 build-only run), gcc -O3 with "
                      f"OpenMP over Step 5's rows, {used} threads",
            "samples": [round(v, 2) for v in multi_s],
            "single_thread": {"value": single, "unit": "pivots/s", "cores": 1,
                              "sample": f"first {k_single} pivots per sample, median of {samples}",
                              "samples": [round(v, 2) for v in single_s],
                              "effective_GBps": round(single * bpp / 1e9, 1),
                              "frac_of_host_triad": round(single * bpp / 1e9 / triad_single, 3)},
            "host": host}


def counter_traffic(name: str, pivots_per_launch: int):
    """HBM bytes per launch from the committed PMC summary
    profiles/<name>_counters.json (FETCH_SIZE and WRITE_SIZE scaled by a
    plain copy of known size), or None when the kernel sources changed since
    the counters were taken or the launch is not the one they were taken on."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{name}_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    h = hashlib.sha256()
    for src in d["kernel_sources"]:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != d["kernel_source_sha256"] or pivots_per_launch != d["pivots"]:
        return None
    return (d["fetch_size_kib"] * d["fetch_scale"] + d["write_size_kib"] * d["write_scale"]) * 1024.0


def traffic_fields(traffic_bytes, avg_ms, algorithmic_bytes):
    """roofline traffic as a rate (GB/s, the unit of `achieved`), per launch,
    and as a ratio to the algorithmic bytes; None fields when unmeasured."""
    if traffic_bytes is None:
        return {"traffic": None, "traffic_GB_per_launch": None, "traffic_over_algorithmic": None}
    return {"traffic": round(traffic_bytes / (avg_ms / 1e3) / 1e9, 1),
            "traffic_GB_per_launch": round(traffic_bytes / 1e9, 1),
            "traffic_over_algorithmic": round(traffic_bytes / algorithmic_bytes, 4)}


def single_schedule(m, n, full_tableau):
    """Best one-LP schedule for a comparison against batching: the LDS
    workgroup when the tableau fits in LDS, else the grid on the tableau form
    the batch uses."""
    from paper_1804_04737_amd import lpdense
    if lpdense.workspace_bytes(m, n) == 0 or full_tableau:
        return lpdense.SCHED_AUTO
    return lpdense.SCHED_GRID_CONDENSED


def batch_cpu_baseline(lps, threads: int):
    """The batched LPs on this host's cores, one LP per thread at a time (the
    serial oracle, whose ctypes calls release the GIL): the batch's reported
    CPU baseline, as the paper's shared-memory machine would run independent
    LPs."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    oracle.solve(*lps[0])  # load the library outside the timed region
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        statuses = list(ex.map(lambda lp: oracle.solve(*lp).status, lps))
    el = time.perf_counter() - t0
    return {"LPs_per_s": round(len(lps) / el, 2), "seconds": round(el, 3), "threads": threads, "kind": "oracle",
            "statuses_optimal": int(sum(1 for x in statuses if x == oracle.OPTIMAL)),
            "sample": f"all {len(lps)} LPs of the batch, full tableau, one thread per LP"}


def batch_summary(args, steps: int, warmup: int):
    """Batched workload: one lp_solve_batch call on 1024 LPs with m, n
    log-uniform in [32, 1024] (seed 0) per step, against solving the same
    resident LPs one lp_solve_dense_ex call at a time on the same stream."""
    import numpy as np
    import torch

    from paper_1804_04737_amd import lpdense, lpgen
    lpdense.load()
    lps = lpgen.batch_lps(args.batch_count, args.batch_lo, args.batch_hi, args.seed)
    pb = lpdense.pack_batch(lps)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    kw = dict(team_size=args.team_size, team_min_bytes=args.team_min_bytes, wave_slots=args.wave_slots,
              full_tableau=args.full_tableau, stream=stream)
    for _ in range(warmup):
        lpdense.solve_batch(pb, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        lpdense.solve_batch(pb, **kw)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    piv = pb.iterations.cpu().numpy()
    st = pb.status.cpu().numpy()
    R = pb.m + 1
    W = pb.n + pb.m + 1 if args.full_tableau else pb.n + 1  # stored columns + RHS
    bytes_step = float(np.sum(piv * 16.0 * R * W))
    lps_s = args.batch_count * steps / el
    log(f"batched: {el * 1e3 / steps:.2f} ms/step, {lps_s:.1f} LPs/s, statuses {np.bincount(st)}")
    # One LP per call, same resident inputs, same stream.
    views = []
    for i in range(pb.count):
        m, n = int(pb.m[i]), int(pb.n[i])
        a0, b0, c0 = int(pb.A_off[i]), int(pb.b_off[i]), int(pb.c_off[i])
        views.append((pb.A[a0:a0 + m * n].view(m, n), pb.b[b0:b0 + m], pb.c[c0:c0 + n]))
    # Each LP on its best single-LP schedule: LDS workgroup if it fits, else the
    # grid on the same tableau form as the batch.
    scheds = [single_schedule(int(pb.m[i]), int(pb.n[i]), args.full_tableau) for i in range(pb.count)]
    for v, sc in list(zip(views, scheds))[:8]:
        lpdense.solve_dense_ex(*v, want_y=False, schedule=sc, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for v, sc in zip(views, scheds):
        lpdense.solve_dense_ex(*v, want_y=False, schedule=sc, stream=stream)
    torch.cuda.synchronize()
    el1 = time.perf_counter() - t0
    single_lps_s = pb.count / el1
    log(f"one at a time: {el1 * 1e3:.1f} ms for {pb.count} LPs, {single_lps_s:.1f} LPs/s")
    cpu = None
    if not getattr(args, "no_cpu_baseline", False):
        host = host_cpu()
        threads = min(host["physical_cores"], host["logical_cpus_allowed"])
        omp_env = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
        cpu = batch_cpu_baseline(lps, min(threads, omp_env) if omp_env > 0 else threads)
        log(f"CPU oracle, {cpu['threads']} threads: {cpu['LPs_per_s']:.1f} LPs/s")
    tr = None
    if (args.batch_count, args.batch_lo, args.batch_hi, args.seed) == (1024, 32, 1024, 0) and not args.full_tableau \
            and (args.team_size, args.team_min_bytes, args.wave_slots) == (0, 0, 0):
        tr = counter_traffic("batch_kernel_batch1024", int(piv.sum()))
    return {"workload": f"batched: {args.batch_count} dense LPs, m and n log-uniform in "
                        f"[{args.batch_lo}, {args.batch_hi}], seed {args.seed}, one lp_solve_batch call per step",
            "hbm_traffic_GBps": None if tr is None else round(tr / (el / steps) / 1e9, 1),
            "hbm_traffic_frac_of_peak": None if tr is None else round(tr / (el / steps) / 1e9 / HBM_PEAK_GBS, 4),
            "LPs_per_s": round(lps_s, 2), "ms_per_step": round(el * 1e3 / steps, 3), "steps": steps,
            "statuses_optimal": int(np.sum(st == lpdense.OPTIMAL)),
            "pivots_per_step": int(piv.sum()), "aggregate_pivots_per_s": round(piv.sum() / (el / steps), 1),
            "effective_GBps": round(bytes_step / (el / steps) / 1e9, 1),
            "one_at_a_time_LPs_per_s": round(single_lps_s, 2),
            "one_at_a_time_effective_GBps": round(bytes_step / el1 / 1e9, 1),
            "speedup_vs_one_at_a_time": round(lps_s / single_lps_s, 2),
            "team_size": args.team_size, "team_min_bytes": args.team_min_bytes,
            "wave_slots": args.wave_slots, "tableau": "full" if args.full_tableau else "condensed",
            "cpu_baseline": cpu, "speedup_vs_cpu_baseline": None if cpu is None else round(lps_s / cpu["LPs_per_s"], 1)}


def batch_bench(args):
    b = batch_summary(args, args.steps, args.warmup)
    out = {
        "metric": METRIC, "value": b["LPs_per_s"], "unit": "LPs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": b["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": b,
    }
    print(json.dumps(out), flush=True)


def serve_summary(args, rates, n_requests: int, n_warmup: int):
    """Served workload: Poisson arrivals of dense LPs (m, n log-uniform in
    [64, 4096], seed-fixed pool) submitted from the host to one lpd_server
    with a footprint budget; per arrival rate, p50/p99 latency (submit to
    result in host memory) and completed LPs/s.  Compared with solving the
    same requests one lp_solve_dense_ex call at a time (host copies included,
    as for the server)."""
    import numpy as np
    import torch

    from paper_1804_04737_amd import lpdense, lpgen
    lpdense.load()
    # Requests live in pinned host memory, as a serving front end would keep them.
    keep = []
    def pinned(a):
        t = torch.from_numpy(a).pin_memory()
        keep.append(t)
        return t.numpy()
    pool = [tuple(pinned(v) for v in lp) for lp in lpgen.batch_lps(args.serve_pool, 64, 4096, args.seed)]
    log(f"pool of {len(pool)} LPs generated (pinned host memory)")
    rng = np.random.default_rng(args.seed + 1)
    picks = [int(v) for v in rng.integers(0, len(pool), size=n_requests)]
    dev = torch.device("cuda")

    # One at a time: host inputs copied in, solved, x copied back, per request.
    stream = torch.cuda.current_stream()
    def one(lp):
        A, b, c = (torch.from_numpy(v).to(dev, non_blocking=False) for v in lp)
        sc = single_schedule(A.shape[0], A.shape[1], args.full_tableau)
        r = lpdense.solve_dense_ex(A, b, c, want_y=False, schedule=sc, stream=stream)
        return r.x.cpu(), int(r.iterations.item())
    def alg_bytes(m, n, piv):
        return 16.0 * (m + 1) * ((n + m + 1) if args.full_tableau else (n + 1)) * piv
    for q in range(min(3, len(pool))):
        one(pool[picks[q]])
    torch.cuda.synchronize()
    n1 = min(len(picks), args.serve_single)
    t0 = time.perf_counter()
    b1 = 0.0
    for q in range(n1):
        _, piv = one(pool[picks[q]])
        b1 += alg_bytes(*pool[picks[q]][0].shape, piv)
    torch.cuda.synchronize()
    el1 = max(time.perf_counter() - t0, 1e-9)
    single_lps_s = n1 / el1 if n1 else float("nan")
    log(f"one at a time: {single_lps_s:.1f} LPs/s over {n1} requests, {b1 / el1 / 1e9:.0f} GB/s effective")

    sweep = []
    n_req = len(picks)
    for rate in rates:
        arr = lpgen.poisson_arrivals(rate, n_req + n_warmup, args.seed + int(rate))
        reqs = [pool[p] for p in rng.integers(0, len(pool), size=n_warmup)] + [pool[p] for p in picks]
        with lpdense.Server(int(args.budget_gb * 1e9), pivots_per_epoch=args.pivots_per_epoch,
                            epoch_bytes_per_wg=int(args.epoch_mb * (1 << 20)),
                            team_bytes_per_wg=int(args.share_kb * 1024),
                            max_resident=args.max_resident, full_tableau=args.full_tableau) as srv:
            done = []
            ids = []
            i = 0
            k_first = w_first = None  # device busy time and wall clock when the timed requests start
            t0 = time.perf_counter()
            while len(done) < len(reqs):
                now = time.perf_counter() - t0
                while i < len(reqs) and arr[i] <= now:
                    if i == n_warmup:
                        k_first, w_first = srv.stats().kernel_seconds, time.perf_counter()
                    ids.append(srv.submit(*reqs[i]))
                    i += 1
                done += srv.poll()
                wait = (arr[i] - (time.perf_counter() - t0)) if i < len(reqs) else 0.0005
                time.sleep(min(max(wait, 0.0), 0.0005))
            st = srv.stats()
            w_last = time.perf_counter()
        # The first requests warm the server up; statistics cover the rest.
        measured = set(ids[n_warmup:])
        bad = [d for d in done if d.status != lpdense.OPTIMAL]
        done = [d for d in done if d.id in measured]
        lat = np.array([d.latency for d in done]) * 1e3
        span = max(d.t_done for d in done) - min(d.t_arrive for d in done)
        gb = sum(alg_bytes(d.m, d.n, d.iterations) for d in done) / 1e9
        row = {"rate_per_s": rate, "requests": len(done), "p50_ms": round(float(np.percentile(lat, 50)), 2),
               "p99_ms": round(float(np.percentile(lat, 99)), 2), "LPs_per_s": round(len(done) / span, 1),
               "effective_GBps": round(gb / span, 1),
               "kernel_busy": round((st.kernel_seconds - k_first) / max(w_last - w_first, 1e-9), 3),
               "admit_host_s": round(st.admit_host_seconds, 3),
               "epochs": int(st.epochs), "peak_GB": round(st.peak_bytes / 1e9, 2), "not_optimal": len(bad)}
        log(f"rate {rate:g}/s: {row}")
        sweep.append(row)
    top = sweep[-1]
    return {"workload": f"served: Poisson arrivals of {n_warmup} warm-up + {len(picks)} timed dense "
                        f"LPs per rate drawn from a pool of "
                        f"{len(pool)} (m, n log-uniform in [64, 4096], seed {args.seed}), footprint budget "
                        f"{args.budget_gb:g} GB, {args.max_resident or 'default'} resident slots, "
                        + (f"{args.pivots_per_epoch} pivots per LP per epoch" if args.pivots_per_epoch > 0
                           else f"pivot budgets sized for {args.epoch_mb:g} MiB per workgroup per epoch"),
            "tableau": "full" if args.full_tableau else "condensed",
            "LPs_per_s_at_top_rate": top["LPs_per_s"],
            "p50_ms_at_top_rate": top["p50_ms"], "p99_ms_at_top_rate": top["p99_ms"],
            "one_at_a_time_LPs_per_s": round(single_lps_s, 2),
            "one_at_a_time_effective_GBps": round(b1 / el1 / 1e9, 1),
            "speedup_vs_one_at_a_time": round(top["LPs_per_s"] / single_lps_s, 2) if n1 else None,
            "sweep": sweep}


def serve_bench(args):
    rates = [float(r) for r in args.serve_rates.split(",")]
    sv = serve_summary(args, rates, args.serve_requests, args.serve_warmup)
    out = {
        "metric": METRIC, "value": sv["LPs_per_s_at_top_rate"], "unit": "LPs/s", "n_gpus": 1, "steps": len(rates),
        "warmup": 0, "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic", "config": sv,
    }
    print(json.dumps(out), flush=True)


def shapes_bench(args):
    """The paper's shape grid: m, n in {256, ..., 8192} (36 shapes), one full
    solve each on the full and on the condensed tableau, with the chosen
    generator (seed fixed).  Reports pivots, ms and pivots/s per shape; the
    paper's observation that more variables than constraints solve faster is
    about wall time, which this splits into pivot count and time per pivot."""
    import torch

    from paper_1804_04737_amd import lpdense, lpgen
    lpdense.load()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    gen = lpgen.paper_lp if args.generator == "paper" else lpgen.dense_lp
    rows = []
    t_all = 0.0
    piv_all = 0
    for m in lpgen.PAPER_SIZES:
        for n in lpgen.PAPER_SIZES:
            A, b, c = gen(m, n, args.seed)
            tA, tb, tc = (torch.from_numpy(v).to(dev) for v in (A, b, c))
            row = {"m": m, "n": n}
            for name, sched in (("full", lpdense.SCHED_AUTO), ("condensed", lpdense.SCHED_GRID_CONDENSED),
                                ("paired", lpdense.SCHED_GRID_PAIRED),
                                ("condensed_paired", lpdense.SCHED_GRID_CONDENSED_PAIRED)):
                lpdense.solve_dense_ex(tA, tb, tc, want_y=False, schedule=sched, stream=stream, max_iter=2)
                s0 = torch.cuda.Event(enable_timing=True)
                s1 = torch.cuda.Event(enable_timing=True)
                s0.record(stream)
                r = lpdense.solve_dense_ex(tA, tb, tc, want_y=False, schedule=sched, stream=stream,
                                           max_iter=2 * (m + n))
                s1.record(stream)
                torch.cuda.synchronize()
                ms = s0.elapsed_time(s1)
                piv = int(r.iterations.item())
                row[f"{name}_ms"] = round(ms, 3)
                row[f"{name}_pivots_per_s"] = round(piv / (ms / 1e3), 1) if ms > 0 else None
                row["pivots"] = piv
                row["status"] = lpdense.STATUS_NAMES[int(r.status.item())]
                if name == "condensed":
                    t_all += ms / 1e3
                    piv_all += piv
            rows.append(row)
            log(json.dumps(row))
            del tA, tb, tc
    out = {
        "metric": METRIC, "value": round(piv_all / t_all, 1), "unit": "pivots/s", "n_gpus": 1,
        "steps": len(rows), "warmup": 0, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"shape grid m, n in {list(lpgen.PAPER_SIZES)}, {args.generator} generator, "
                               f"seed {args.seed}, one solve per shape and schedule (at most 2 (m+n) "
                               f"pivots); value = all "
                               f"condensed pivots / all condensed time", "shapes": rows},
    }
    print(json.dumps(out), flush=True)


def copy_calibration():
    """A plain 1 GiB device-to-device copy: its FETCH_SIZE / WRITE_SIZE
    readings calibrate the HBM byte counters of the solve kernels."""
    import torch
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    log("copied 1 GiB for counter calibration")


def small_lp_summary(args, calls: int = 400):
    """The 64 x 64 LP (seed 0, 13 pivots): back-to-back lp_solve_dense calls
    on one stream with resident inputs and outputs (the LDS-resident
    workgroup schedule the library picks for it), timed with HIP events."""
    import torch

    from paper_1804_04737_amd import lpdense, lpgen
    A, b, c = lpgen.dense_lp(64, 64, 0)
    dev = torch.device("cuda:0")
    tA, tb, tc = (torch.from_numpy(v).to(dev) for v in (A, b, c))
    stream = torch.cuda.current_stream()
    out = {"workload": "dense LP m = n = 64, seed 0, full solve, lp_solve_dense (auto schedule)"}
    x = torch.empty(64, dtype=torch.float64, device=dev)
    obj = torch.empty(1, dtype=torch.float64, device=dev)
    st = torch.empty(1, dtype=torch.int32, device=dev)
    r = lpdense.solve_dense_ex(tA, tb, tc, stream=stream)
    torch.cuda.synchronize()
    piv = int(r.iterations.item())
    for _ in range(20):
        lpdense.solve_dense(tA, tb, tc, x, obj, st, stream=stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(calls):
        lpdense.solve_dense(tA, tb, tc, x, obj, st, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    us = e0.elapsed_time(e1) * 1e3 / calls
    out.update({"pivots": piv, "status": lpdense.STATUS_NAMES[int(st.item())], "calls": calls,
                "us_per_solve": round(us, 2), "pivots_per_s": round(piv / (us * 1e-6), 1),
                "solves_per_s": round(1e6 / us, 1), "host_us_per_call": round(wall * 1e6 / calls, 2)})
    log(f"64x64: {out}")
    return out


CONFIG_SHAPES = [(4096, 4096), (8192, 1024), (1024, 8192), (2048, 8192)]


def shapes_summary(args, reps: int = 2):
    """4096 x 4096 and the primal-like / dual-like shapes 8192 x 1024,
    1024 x 8192 and 2048 x 8192 (seed 0, full solves) on the four grid
    schedules: pivots, ms per solve, pivots/s, GB/s of each schedule's own
    bytes per sweep and its fraction of 8 TB/s (HIP events, mean of `reps`
    solves after one warm-up solve)."""
    import torch

    from paper_1804_04737_amd import lpdense, lpgen
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    rows = []
    for m, n in CONFIG_SHAPES:
        A, b, c = lpgen.dense_lp(m, n, args.seed)
        tA, tb, tc = (torch.from_numpy(v).to(dev) for v in (A, b, c))
        row = {"m": m, "n": n}
        for name, sched, cols, paired in (("full", lpdense.SCHED_AUTO, n + m + 1, False),
                                          ("condensed", lpdense.SCHED_GRID_CONDENSED, n + 1, False),
                                          ("paired", lpdense.SCHED_GRID_PAIRED, n + m + 1, True),
                                          ("condensed_paired", lpdense.SCHED_GRID_CONDENSED_PAIRED, n + 1, True)):
            lpdense.solve_dense_ex(tA, tb, tc, want_y=False, schedule=sched, stream=stream)
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
            rs = []
            for e0, e1 in ev:
                e0.record(stream)
                rs.append(lpdense.solve_dense_ex(tA, tb, tc, want_y=False, schedule=sched, stream=stream))
                e1.record(stream)
            torch.cuda.synchronize()
            ms = sum(e0.elapsed_time(e1) for e0, e1 in ev) / reps
            piv = int(rs[0].iterations.item())
            sweeps = (piv + 1) // 2 if paired else piv
            gbs = 16.0 * (m + 1) * cols * sweeps / (ms / 1e3) / 1e9
            row["pivots"] = piv
            row["status"] = lpdense.STATUS_NAMES[int(rs[0].status.item())]
            row[name] = {"ms_per_solve": round(ms, 3), "pivots_per_s": round(piv / (ms / 1e3), 1),
                         "GBps": round(gbs, 1), "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)}
        log(f"shape {m}x{n}: {row}")
        rows.append(row)
        del tA, tb, tc
    return {"workload": "dense LPs (generator of the 64x64 and 8192x8192 LPs), seed 0, full solves; "
                        "GBps counts each schedule's own bytes per sweep: 16 (m+1) W with W = n+m+1 (full) "
                        "or n+1 (condensed), one sweep per pivot or per two (paired)",
            "rows": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--m", type=int, default=8192)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--max-iter", type=int, default=-1, help="pivot cap per solve (-1: solve to the end)")
    ap.add_argument("--grid-blocks", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=24.0,
                    help="CPU work of the oracle baseline (half multi-threaded, half single-threaded)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-condensed", action="store_true",
                    help="dense: skip the extra timing of the same LP on the condensed tableau")
    ap.add_argument("--no-extras", action="store_true",
                    help="dense: skip the 64x64 LP, the shape sweep, the batched and the served workloads")
    ap.add_argument("--extra-serve-rates", default="100,400,1000",
                    help="dense run's served workload: arrival rates (LPs/s), the last past saturation")
    ap.add_argument("--extra-serve-requests", type=int, default=500, help="dense run: timed requests per rate")
    ap.add_argument("--extra-serve-warmup", type=int, default=50, help="dense run: untimed requests per rate")
    ap.add_argument("--extra-batch-steps", type=int, default=5, help="dense run: timed lp_solve_batch calls")
    ap.add_argument("--phases", action="store_true",
                    help="after the timed steps, run one more solve with per-phase device timestamps")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 1 GiB device-to-device (reference kernel for HBM byte counters)")
    ap.add_argument("--workload", choices=["dense", "batch", "serve", "shapes"], default="dense")
    ap.add_argument("--generator", choices=["dense", "paper"], default="dense",
                    help="dense / shapes: the main generator, or the paper-style one (zeros in A, b = A x0)")
    ap.add_argument("--schedule", choices=["auto", "condensed", "paired", "condensed_paired"], default="auto",
                    help="dense: full tableau (auto: grid for large LPs), the condensed tableau "
                         "(nonbasic columns only), or two pivots per sweep of either; "
                         "all give bitwise-identical results")
    ap.add_argument("--serve-rates", default="100,200,500,1000,2000,5000", help="serve: arrival rates (LPs/s)")
    ap.add_argument("--serve-requests", type=int, default=2000, help="serve: timed requests per rate")
    ap.add_argument("--serve-warmup", type=int, default=100, help="serve: untimed requests before them")
    ap.add_argument("--serve-pool", type=int, default=48, help="serve: distinct LPs the requests draw from")
    ap.add_argument("--serve-single", type=int, default=100, help="serve: requests timed one at a time")
    ap.add_argument("--pivots-per-epoch", type=int, default=0,
                    help="serve: pivot budget per LP per launch (0: sized per LP from --epoch-mb)")
    ap.add_argument("--epoch-mb", type=float, default=256.0,
                    help="serve: tableau MiB each workgroup streams per launch (sizes the pivot budgets)")
    ap.add_argument("--max-resident", type=int, default=0, help="serve: resident slots (0: library default)")
    ap.add_argument("--share-kb", type=float, default=0,
                    help="serve: least tableau KiB per workgroup of a team (0: library default)")
    ap.add_argument("--budget-gb", type=float, default=200.0, help="serve: footprint budget (1e9 bytes)")
    ap.add_argument("--batch-count", type=int, default=1024)
    ap.add_argument("--batch-lo", type=int, default=32, help="batch: smallest m and n")
    ap.add_argument("--batch-hi", type=int, default=1024, help="batch: largest m and n")
    ap.add_argument("--wave-slots", type=int, default=0, help="batch: wave-per-instance slots (0: autotune table)")
    ap.add_argument("--full-tableau", action="store_true",
                    help="batch / serve: grid walks on the full tableau instead of the condensed one")
    ap.add_argument("--team-size", type=int, default=0, help="batch: workgroups per team (0: autotune table)")
    ap.add_argument("--team-min-bytes", type=int, default=0, help="batch: team threshold (0: autotune table)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported: the benchmark runs on one GPU only "
              f"(one LP per GPU; sharding over several GPUs is not built).", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration()
    if args.workload == "batch":
        return batch_bench(args)
    if args.workload == "serve":
        return serve_bench(args)
    if args.workload == "shapes":
        return shapes_bench(args)

    import numpy as np
    import torch

    from paper_1804_04737_amd import lpdense, lpgen

    lpdense.load()
    dev = torch.device("cuda:0")
    m, n = args.m, args.n
    log(f"generating {m}x{n} LP seed {args.seed} ({args.generator} generator)")
    A, b, c = (lpgen.paper_lp if args.generator == "paper" else lpgen.dense_lp)(m, n, args.seed)
    tA = torch.from_numpy(A).to(dev)
    tb = torch.from_numpy(b).to(dev)
    tc = torch.from_numpy(c).to(dev)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()

    sched = {"auto": lpdense.SCHED_AUTO, "condensed": lpdense.SCHED_GRID_CONDENSED,
             "paired": lpdense.SCHED_GRID_PAIRED,
             "condensed_paired": lpdense.SCHED_GRID_CONDENSED_PAIRED}[args.schedule]

    def step():
        return lpdense.solve_dense_ex(tA, tb, tc, max_iter=args.max_iter, schedule=sched,
                                      grid_blocks=args.grid_blocks, want_y=True, stream=stream)

    for w in range(args.warmup):
        log(f"warmup {w}")
        r = step()
        torch.cuda.synchronize()
        log(f"warmup {w} done: status={lpdense.STATUS_NAMES[int(r.status.item())]} "
            f"pivots={int(r.iterations.item())} z={float(r.obj.item())!r}")

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    results = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        starts[k].record(stream)
        results.append(step())
        ends[k].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    pivots = [int(r.iterations.item()) for r in results]
    statuses = [int(r.status.item()) for r in results]
    ev_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    total_piv = sum(pivots)
    log(f"timed {args.steps} steps in {elapsed:.3f} s; pivots per step {pivots}; event ms {ev_ms}")

    # Algorithmic bytes: the stored tableau read and written once per sweep
    # (the full tableau, or only the nonbasic columns and the RHS).  A sweep
    # does one pivot, or two on the paired schedule: ceil(pivots / 2) sweeps
    # there, since a sweep takes one pivot only where the solve then ends.
    R, W = m + 1, (n + 1 if args.schedule in ("condensed", "condensed_paired") else n + m + 1)
    bytes_per_sweep = 16.0 * R * W
    sweeps = [(p + 1) // 2 if args.schedule in ("paired", "condensed_paired") else p for p in pivots]
    bytes_per_pivot = bytes_per_sweep * sweeps[0] / max(pivots[0], 1)
    avg_ms = sum(ev_ms) / len(ev_ms)
    achieved = bytes_per_sweep * (sum(sweeps) / args.steps) / (avg_ms / 1e3) / 1e9
    headline_lp = (m, n, args.seed) == (8192, 8192, 0) and args.generator == "dense" and args.max_iter < 0
    counters = {"auto": "grid_solve_kernel_dense8192", "condensed": "grid_solve_kernel_condensed_dense8192",
                "paired": "grid_solve_kernel_paired_dense8192",
                "condensed_paired": "grid_solve_kernel_condensed_paired_dense8192"}
    traffic = counter_traffic(counters[args.schedule], pivots[0]) if headline_lp else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                **traffic_fields(traffic, avg_ms, bytes_per_sweep * sweeps[0])}

    phases = None
    if args.phases:
        K = max(pivots)
        r = lpdense.solve_dense_ex(tA, tb, tc, max_iter=args.max_iter, grid_blocks=args.grid_blocks,
                                   phase_cap=K, schedule=sched, stream=stream)
        torch.cuda.synchronize()
        it = int(r.iterations.item())
        if r.phase_ticks is not None and it > 2:
            t = r.phase_ticks.cpu().numpy()[1:it].astype(np.int64)
            t = t[t[:, 0] > 0]  # paired schedule: one entry per sweep, at its first pivot
            d = np.median(np.diff(t[:, :7], axis=1), axis=0) * 10e-3  # us (100 MHz clock)
            tot = float(np.median(t[:, 6] - t[:, 0])) * 10e-3
            phases = {"us_per_sweep_median": round(tot, 2), "pricing": round(d[0], 2),
                      "update_wg0": round(d[1], 2), "wait_last_wg": round(d[2], 2),
                      "release": round(d[3], 2), "detect": round(d[4], 2), "reduce": round(d[5], 2)}
            if args.schedule in ("paired", "condensed_paired"):
                # Entry 7: end of the wait at the pair's publication barrier
                # (part of the update share above).
                phases["pair_barrier_wait"] = round(float(np.median(t[:, 7] - t[:, 1])) * 10e-3, 2)
            log(f"phases (median us/pivot): {phases}")

    # Same LP on the condensed tableau and with two pivots per sweep
    # (bitwise-identical results, fewer bytes per pivot): reported beside the
    # full-tableau figures.
    def other_schedule(sc, bytes_per_sweep_sc, sweeps_of, counter_name):
        lpdense.solve_dense_ex(tA, tb, tc, max_iter=args.max_iter, schedule=sc, want_y=False, stream=stream)
        cs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
        ce = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
        rs = []
        for k in range(args.steps):
            cs[k].record(stream)
            rs.append(lpdense.solve_dense_ex(tA, tb, tc, max_iter=args.max_iter, schedule=sc, want_y=False,
                                             stream=stream))
            ce[k].record(stream)
        torch.cuda.synchronize()
        cms = sum(x.elapsed_time(y) for x, y in zip(cs, ce)) / args.steps
        cpiv = int(rs[0].iterations.item())
        same = all(bool(torch.equal(r.x.view(torch.int64), results[0].x.view(torch.int64))) for r in rs)
        alg = bytes_per_sweep_sc * sweeps_of(cpiv)
        tr = counter_traffic(counter_name, cpiv) if headline_lp else None
        return {"pivots_per_s": round(cpiv / (cms / 1e3), 2), "ms_per_solve": round(cms, 3),
                "pivots_per_step": cpiv, "sweeps_per_step": sweeps_of(cpiv),
                "bytes_per_sweep": int(bytes_per_sweep_sc),
                "stored_bytes_GBps": round(alg / (cms / 1e3) / 1e9, 1),
                "frac_of_hbm_peak": round(alg / (cms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                **traffic_fields(tr, cms, alg),
                "x_bitwise_equal_to_full_tableau": same}

    condensed = paired = condensed_paired = None
    if args.schedule == "auto" and not args.no_condensed:
        condensed = other_schedule(lpdense.SCHED_GRID_CONDENSED, 16.0 * (m + 1) * (n + 1), lambda p: p,
                                   counters["condensed"])
        log(f"condensed tableau: {condensed}")
        paired = other_schedule(lpdense.SCHED_GRID_PAIRED, 16.0 * (m + 1) * (n + m + 1), lambda p: (p + 1) // 2,
                                counters["paired"])
        log(f"two pivots per sweep: {paired}")
        condensed_paired = other_schedule(lpdense.SCHED_GRID_CONDENSED_PAIRED, 16.0 * (m + 1) * (n + 1),
                                          lambda p: (p + 1) // 2, counters["condensed_paired"])
        log(f"two pivots per sweep of the condensed tableau: {condensed_paired}")

    extras = {}
    if not args.no_extras:
        # The rest of the metric on the same GPU: the 64 x 64 LP, the shape
        # sweep, the batched workload and the served one.
        del results
        extras["small_lp"] = small_lp_summary(args)
        extras["shapes"] = shapes_summary(args)
        extras["batch"] = batch_summary(args, args.extra_batch_steps, 1)
        extras["serve"] = serve_summary(args, [float(r) for r in args.extra_serve_rates.split(",")],
                                        args.extra_serve_requests, args.extra_serve_warmup)

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline(m, n, args.seed, args.generator, args.cpu_seconds)

    out = {
        "metric": METRIC,
        "value": round(total_piv / elapsed, 2),
        "unit": "pivots/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"dense LP max c^T x, Ax<=b, x>=0, m={m}, n={n}, seed {args.seed}, "
                               + ("paper-style generator, " if args.generator == "paper" else "")
                               + "full solve from the slack basis (Dantzig, lowest-index ties)"
                               + {"auto": "", "condensed": "; condensed tableau (nonbasic columns only)",
                                  "paired": "; two pivots per sweep of the full tableau",
                                  "condensed_paired": "; two pivots per sweep of the condensed tableau"}[args.schedule],
                   "schedule": args.schedule,
                   "m": m, "n": n, "pivots_per_step": pivots[0],
                   "status": lpdense.STATUS_NAMES[statuses[0]],
                   "bytes_per_pivot": int(bytes_per_pivot), "sweeps_per_step": sweeps[0],
                   "max_iter": args.max_iter, "phases_us": phases, "condensed_tableau": condensed,
                   "two_pivots_per_sweep": paired, "condensed_two_pivots_per_sweep": condensed_paired},
        "roofline": roofline,
        "cpu_baseline": cpu,
        **extras,
    }
    print(json.dumps(out), flush=True)
    # Orderly teardown before the interpreter exits: no kernel in flight and
    # no cached device memory left to torch's exit path.
    del tA, tb, tc
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


if __name__ == "__main__":
    if len(sys.argv) == 3 and sys.argv[1] == "--cpu-baseline-child":
        _cpu_baseline_child(sys.argv[2])
    else:
        main()
