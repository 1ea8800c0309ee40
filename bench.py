"""Benchmark: committed spin-updates per second on one MI355X.

A step is one pass of the whole hot path over the 4096x4096 critical lattice:
initial draws (aca_init) and the conservative sweep to the horizon T = 200
(aca_advance), i.e. about 3.4e9 applied arrivals.  The lattice buffers are
allocated in HBM before the timed region; the final state is read back and
checked against the oracle's digest after it.

Prints one JSON line.  Besides the contract fields it carries
  roofline      the visit kernel: algorithmic bytes or per-arrival operations
                per launch over the launch time measured with HIP events on the
                launching stream (inside the library), against MI355X peaks;
  other_configs the 64^2 and 256^3 lattices (automatic schedules): time per
                advance, arrival rate, arithmetic-bound fraction, bit-exactness;
  cpu_baseline  the serial oracle timed on a bounded sample of the same workload
                on one host core, the host's CPU model and core count, and an
                all-core aggregate (one batch lattice per worker process);
  batched       the 512-lattice workload (sides log-uniform in [32, 1024],
                uneven temperatures and horizons): one batch advance against the
                plain path of one init + advance per lattice on one stream, in
                jobs/s, with the speedup;
  served        the job stream (80% 2D up to 2048^2, 20% 3D up to 128^3, both
                rules, horizons up to 1000) through the job server: first all
                jobs at once (capacity in jobs/s), then Poisson arrivals at 0.7
                of that capacity, with p50/p99 of result-on-host minus arrival;
                the same jobs through the plain path (one init + advance per
                job, in arrival order) for the served-vs-plain speedup, and the
                2D and 3D jobs served apart.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Plain VALU issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one wave64
# instruction every 4 cycles per SIMD; binary64 add/mul run at this rate).
VALU_LANE_OPS_PER_S = 256 * 4 * 16 * 2.4e9
# Issue slots one applied arrival needs at minimum on gfx950: Philox4x32-10 is
# 20 v_mad_u64_u32 (half rate, 2 slots each) and 20 v_bitop3_b32; -ln u is 48
# binary64 slots (16 mul, 16 add, the quotient's reciprocal -- quarter rate --
# with its Newton steps and correction, conversions) and 11 integer ones; flip
# test and clock update 8.
SLOTS_PER_EVENT = 40 + 20 + 48 + 11 + 8


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def digest(s, t, n):
    return (hashlib.sha256(s.tobytes()).hexdigest(),
            hashlib.sha256(t.astype("<f8").tobytes()).hexdigest(),
            hashlib.sha256(n.astype("<u4").tobytes()).hexdigest())


VISIT_SOURCES = ("aca_device.h", "aca_internal.h", "aca_region.h", "aca_visit_fast.hip")


def kernel_source_digest() -> str:
    """SHA-256 over the sources the tile-visit kernel of the large lattices is
    compiled from."""
    csrc = os.path.join(ROOT, "paper_cs_0502039_amd", "csrc")
    h = hashlib.sha256()
    for name in VISIT_SOURCES:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic(workload: str, tuning: dict):
    """HBM bytes per visit launch from the committed counter summary
    (profiles/traffic_<workload>.json, FETCH_SIZE + WRITE_SIZE scaled by a copy
    kernel's readings), or None when it is missing, the kernels changed since,
    or the counters were taken with other tiles, ghosts or block size (a
    launch's loads and merges depend on those, not on the rounds per visit)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        doc = json.load(f)
    if doc.get("kernel_source_sha256") != kernel_source_digest():
        return None
    for entry in doc.get("entries", []):
        prof = entry.get("tuning", {})
        if all(list(prof.get(k, [])) == list(tuning.get(k, [])) for k in ("tile", "ghost")) and \
                prof.get("block") == tuning.get("block"):
            return entry["hbm_bytes_per_launch"]
    return None


def copy_calibration(nbytes: int = 1 << 31) -> None:
    """A plain device copy of known size, for scaling FETCH_SIZE / WRITE_SIZE."""
    import torch
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    log(f"copy calibration: {nbytes} bytes read and {nbytes} bytes written")


def host_cpu() -> dict:
    """The host's CPU model and the cores this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "usable_cores": len(os.sched_getaffinity(0)),
            "os_cpu_count": os.cpu_count()}


def cpu_baseline(params: dict, T_sample: float) -> dict:
    import oracle
    log(f"cpu_baseline: oracle on {params['L']} to T={T_sample}")
    t0 = time.time()
    s, t, n = oracle.init(params)
    t1 = time.time()
    ev, _ = oracle.run(params, T_sample, s, t, n)
    t2 = time.time()
    rate = ev / (t2 - t1)
    return {"value": rate, "unit": "spin-updates/s", "cores": 1, "kind": "oracle",
            "host": host_cpu(),
            "sample": (f"{params['L'][0]}^{params['dim']} lattice seed {params['seed']}, "
                       f"binary-heap oracle from the initial state to T={T_sample} "
                       f"({ev} arrivals in {t2 - t1:.1f} s; init {t1 - t0:.1f} s not "
                       f"counted), one thread")}


# arrivals per worker in the all-core sample (about 10 s of one core each)
AGGREGATE_ARRIVALS = 2.0e7


def _oracle_item(params):
    import oracle
    t0 = time.time()
    s, t, n = oracle.init(params)
    ev, _ = oracle.run(params, params["T"], s, t, n)
    return ev, time.time() - t0


def cpu_aggregate_main(workers: int) -> None:
    """All-core oracle on the 512-lattice workload (runs in its own interpreter,
    which never touches the GPU): the first `workers` lattices, one per worker
    process, each to min(T, the horizon of about AGGREGATE_ARRIVALS arrivals)."""
    from multiprocessing import Pool
    from paper_cs_0502039_amd import workloads
    import oracle
    oracle.lib()
    items = []
    for p in workloads.batch_512()[:workers]:
        n = p["L"][0] * p["L"][1]
        items.append(dict(p, T=min(p["T"], AGGREGATE_ARRIVALS / n)))
    t0 = time.time()
    with Pool(workers) as pool:
        res = pool.map(_oracle_item, items)
    wall = time.time() - t0
    events = sum(r[0] for r in res)
    print(json.dumps({"events": events, "wall_s": wall, "workers": workers,
                      "per_worker_rate": [r[0] / r[1] for r in res],
                      "sides": [p["L"][0] for p in items],
                      "horizons": [p["T"] for p in items]}), flush=True)


def cpu_aggregate(max_workers: int = 16) -> dict:
    """The all-core leg of the CPU baseline, in a child interpreter."""
    import subprocess
    workers = max(1, min(max_workers, len(os.sched_getaffinity(0))))
    log(f"cpu_baseline: all-core oracle aggregate, {workers} workers")
    res = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-aggregate-only",
                          str(workers)], capture_output=True, text=True, timeout=600)
    if res.returncode != 0:
        return {"error": res.stderr[-500:]}
    doc = json.loads(res.stdout.strip().splitlines()[-1])
    return {"value": doc["events"] / doc["wall_s"], "unit": "spin-updates/s",
            "cores": workers, "kind": "oracle",
            "per_core": doc["events"] / doc["wall_s"] / workers,
            "sample": (f"the first {workers} lattices of the 512-lattice workload (sides "
                       f"{min(doc['sides'])}-{max(doc['sides'])}), one per worker process, "
                       f"each to min(T, {AGGREGATE_ARRIVALS:.0e} / N): {doc['events']} "
                       f"arrivals in {doc['wall_s']:.1f} s wall")}


def bench_batched(steps: int, warmup: int, autotune: bool = True) -> dict:
    """Batched vs plain on the 512-lattice workload.  With autotune the first
    warm-up pass lets the batch tuner pick the 2D schedule on the workload itself
    (the tuner advances the real lattices, so that pass still ends exact)."""
    import torch
    from paper_cs_0502039_amd import aca, workloads
    cases = workloads.batch_512()
    lats = [aca.Lattice(p) for p in cases]
    T = [p["T"] for p in cases]
    batch = aca.Batch(len(cases))
    log(f"batched: {len(cases)} lattices, {sum(l.n for l in lats)} cells")

    def one_batched():
        for l in lats:
            l.init()
        batch.advance(lats, T)

    tune = None
    if autotune:
        for l in lats:
            l.init()
        tune = batch.tune(lats, T, 2, frac=0.03)
        batch.advance(lats, T)
        log(f"batched: autotuned 2D schedule {tune['tuning']} "
            f"(rates per ms {[round(r) for r in tune['rates_per_ms']]})")
    for _ in range(warmup):
        one_batched()
    torch.cuda.synchronize()
    k0 = batch.stats()
    t0 = time.perf_counter()
    for _ in range(steps):
        one_batched()
    torch.cuda.synchronize()
    dt_b = (time.perf_counter() - t0) / steps
    k1 = batch.stats()
    events = (k1["events"] - k0["events"]) // steps
    log(f"batched: {dt_b * 1e3:.1f} ms per pass, kernel "
        f"{(k1['kernel_ms'] - k0['kernel_ms']) / steps:.1f} ms")
    bit_exact = None
    gold_path = os.path.join(ROOT, "tests", "golden", "batch_512.json")
    if os.path.exists(gold_path):
        with open(gold_path) as f:
            gold = json.load(f)["items"]
        bit_exact = all(
            g["params"] == p and digest(*l.read()) == (g["sha256_s"], g["sha256_t"],
                                                       g["sha256_n"])
            for g, p, l in zip(gold, cases, lats))
        log(f"batched: bit-exact vs oracle digests: {bit_exact}")
    # plain path: one init + advance per lattice, one after another
    small = aca.Lattice(workloads.lattice(2, (64, 64), 0.4, T=2.0))
    small.init().advance(2.0)
    small.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for l, t in zip(lats, T):
        l.init().advance(t)
    torch.cuda.synchronize()
    dt_p = time.perf_counter() - t0
    log(f"plain: {dt_p * 1e3:.1f} ms per pass")
    tuning_2d = batch.tuning(2)
    batch.close()
    for l in lats:
        l.close()
    return {"workload": "batch_512", "lattices": len(cases), "events": events,
            "ms_batched": dt_b * 1e3, "ms_plain": dt_p * 1e3,
            "jobs_per_s": len(cases) / dt_b, "plain_jobs_per_s": len(cases) / dt_p,
            "speedup": dt_p / dt_b, "spin_updates_per_s": events / dt_b,
            "plain_spin_updates_per_s": events / dt_p, "bit_exact": bit_exact,
            "tuning_2d": tuning_2d, "autotune": tune, "steps": steps}


def serve(jobs, arena_bytes: int, max_jobs: int, budget_ms: float, arrivals=None):
    """Drive the job server; arrivals[i] is job i's arrival in seconds after the
    start (None: all at once).  Returns (latencies s, wall s, events, stats)."""
    from paper_cs_0502039_amd import aca
    server = aca.Server(arena_bytes, max_jobs=max_jobs)
    n = len(jobs)
    order = list(range(n)) if arrivals is None else sorted(range(n), key=lambda i: arrivals[i])
    t_arr = [0.0] * n if arrivals is None else list(arrivals)
    ids = {}
    lat = [0.0] * n
    done = 0
    nxt = 0
    t0 = time.perf_counter()
    while done < n:
        now = time.perf_counter() - t0
        while nxt < n and t_arr[order[nxt]] <= now:
            i = order[nxt]
            ids[server.submit(jobs[i])] = i
            nxt += 1
        q, r = server.load()
        if q == 0 and r == 0:
            # idle until the next arrival
            wait = t_arr[order[nxt]] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(min(wait, 0.0005))
            continue
        for job in server.step(budget_ms):
            server.read(job)
            lat[ids[job]] = time.perf_counter() - t0 - t_arr[ids[job]]
            server.release(job)
            done += 1
    wall = time.perf_counter() - t0
    st = server.stats()
    server.close()
    return lat, wall, st


def bench_served(arena_gib: float, max_jobs: int, budget_ms: float, count: int) -> dict:
    import numpy as np
    from paper_cs_0502039_amd import workloads
    stream = workloads.served_stream(count=count, rate_jobs_per_s=1.0)
    jobs = [{k: v for k, v in j.items() if k not in ("t_arrive", "id")} for j in stream]
    unit_arrivals = [j["t_arrive"] for j in stream]       # Poisson, rate 1 per second
    arena = int(arena_gib * (1 << 30))
    log(f"served: {count} jobs, arena {arena_gib} GiB, {max_jobs} slots, "
        f"step budget {budget_ms} ms")
    # warm-up: a few jobs through a small server
    serve(jobs[:4], arena, max_jobs, budget_ms)
    _, wall_c, st_c = serve(jobs, arena, max_jobs, budget_ms)
    capacity = count / wall_c
    rho = 0.7 * capacity
    log(f"served: capacity {capacity:.1f} jobs/s ({st_c['events'] / wall_c:.3e} "
        f"spin-updates/s); open loop at {rho:.1f} jobs/s")
    arrivals = [t / rho for t in unit_arrivals]
    lat, wall, st = serve(jobs, arena, max_jobs, budget_ms, arrivals)
    lat_ms = np.array(lat) * 1e3
    # the same jobs served per dimension alone: where the device time goes
    by_dim = {}
    for dim in (2, 3):
        sub = [j for j in jobs if j["dim"] == dim]
        _, wall_d, st_d = serve(sub, arena, max_jobs, budget_ms)
        by_dim[f"{dim}d"] = {"jobs": len(sub), "served_s": wall_d,
                             "spin_updates": st_d["events"],
                             "spin_updates_per_s": st_d["events"] / wall_d}
    plain = bench_served_plain(jobs)
    log(f"served: plain path {plain['jobs_per_s']:.1f} jobs/s; served capacity "
        f"{capacity:.1f} jobs/s ({capacity / plain['jobs_per_s']:.2f}x)")
    return {"workload": "served_stream", "jobs": count, "arena_gib": arena_gib,
            "max_jobs": max_jobs, "step_budget_ms": budget_ms,
            "capacity_jobs_per_s": capacity,
            "plain_jobs_per_s": plain["jobs_per_s"],
            "speedup_vs_plain": capacity / plain["jobs_per_s"],
            "plain": plain, "by_dim": by_dim,
            "capacity_spin_updates_per_s": st_c["events"] / wall_c,
            # per server step of the capacity run: the persistent visits' device
            # time, and the rest of the step (admission, pack/open/unpack
            # launches, copies, the host's wait) -- the most that capturing a
            # step's launches in a graph could save
            "capacity_steps": st_c["steps"],
            "capacity_kernel_ms_per_step": st_c["kernel_ms"] / max(1, st_c["steps"]),
            "capacity_other_ms_per_step": (st_c["device_ms"] - st_c["kernel_ms"])
            / max(1, st_c["steps"]),
            "rho_jobs_per_s": rho, "jobs_per_s": count / wall,
            "spin_updates_per_s": st["events"] / wall,
            "p50_ms": float(np.percentile(lat_ms, 50)),
            "p99_ms": float(np.percentile(lat_ms, 99)),
            "max_ms": float(lat_ms.max()), "mean_ms": float(lat_ms.mean()),
            "events": st["events"], "steps": st["steps"],
            "arena_peak_gib": st["arena_peak"] / (1 << 30), "queued_peak": st["queued_peak"]}


def bench_config(name: str, steps: int = 3) -> dict:
    """One of the other single-lattice configurations (64^2 to T = 100, 256^3 to
    T = 100) with the automatic schedule: best wall time per advance of several,
    arrivals per second, the visit kernel's fraction of the arithmetic bound, and
    the final state against the oracle's digest."""
    import torch
    from paper_cs_0502039_amd import aca, workloads
    params = getattr(workloads, name)()
    lat = aca.Lattice(params)
    lat.init().advance(params["T"])
    best = None
    for _ in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.init().advance(params["T"])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    st = lat.stats()
    out = {"workload": name, "ms_per_advance": best * 1e3, "events": st["events"],
           "spin_updates_per_s": st["events"] / best, "launches": st["launches"],
           "kernel_ms_per_launch": st["kernel_ms"] / st["launches"],
           "alu_frac": st["events"] / (st["kernel_ms"] / 1e3)
           / (VALU_LANE_OPS_PER_S / SLOTS_PER_EVENT),
           "tuning": lat.tuning()}
    # measured HBM bytes per launch (profiles/traffic_<name>.json) while the
    # kernels and the schedule match the counters, else None
    traffic = measured_traffic(name, lat.tuning())
    out["traffic_bytes_per_launch"] = traffic
    if traffic is not None:
        out["traffic_tb_per_s"] = traffic / (out["kernel_ms_per_launch"] / 1e3) / 1e12
    gold_path = os.path.join(ROOT, "tests", "golden", f"{name}.json")
    if os.path.exists(gold_path):
        with open(gold_path) as f:
            gold = json.load(f)
        out["bit_exact"] = digest(*lat.read()) == (gold["sha256_s"], gold["sha256_t"],
                                                   gold["sha256_n"]) \
            and gold["events"] == st["events"]
    lat.close()
    log(f"{name}: {best * 1e3:.2f} ms per advance, bit-exact {out.get('bit_exact')}")
    return out


def bench_served_plain(jobs) -> dict:
    """The plain path on the served mix: for each job in arrival order, its own
    state buffers, one aca_init + aca_advance on one stream, and the result read
    to the host, one job after another."""
    import torch
    from paper_cs_0502039_amd import aca
    warm = aca.Lattice(dict(jobs[0], L=[32] * jobs[0]["dim"]))
    warm.init().advance(1.0)
    warm.close()
    torch.cuda.synchronize()
    per_dim = {2: [0, 0.0, 0], 3: [0, 0.0, 0]}
    t0 = time.perf_counter()
    for p in jobs:
        t1 = time.perf_counter()
        lat = aca.Lattice(p)
        lat.init().advance(p["T"])
        lat.read()
        ev = lat.stats()["events"]
        lat.close()
        d = per_dim[p["dim"]]
        d[0] += 1
        d[1] += time.perf_counter() - t1
        d[2] += ev
    wall = time.perf_counter() - t0
    return {"jobs": len(jobs), "wall_s": wall, "jobs_per_s": len(jobs) / wall,
            "spin_updates_per_s": sum(d[2] for d in per_dim.values()) / wall,
            "by_dim": {f"{k}d": {"jobs": v[0], "s": v[1], "spin_updates": v[2]}
                       for k, v in per_dim.items()}}


def bench_lag(lags, T: float = 50.0, frame_dt: float = 5.0) -> dict:
    """The bounded-lag experiment (Section 4, efficiency against the lag bound)
    on the 4096^2 critical lattice to T = 50: arrivals per second, launches and
    the fraction of enabling tests that found an enabled cell, per lag bound;
    plus the cost of writing output frames every frame_dt."""
    import torch
    from paper_cs_0502039_amd import aca, workloads
    params = workloads.square_4096()
    lat = aca.Lattice(params)
    lat.init().advance(T)           # warm-up
    rows = []
    for lag in lags:
        lat.set_lag(lag)
        lat.init()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.advance(T)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = lat.stats()
        rows.append({"lag": lag if lag > 0 else None, "ms": dt * 1e3,
                     "spin_updates_per_s": st["events"] / dt, "launches": st["launches"],
                     "enabled_per_check": (st["events"] + st["ghost_events"])
                     / max(1, st["cell_checks"])})
        log(f"lag {lag}: {dt * 1e3:.1f} ms, {st['launches']} launches")
    lat.set_lag(0.0)
    nframes = int(T / frame_dt)
    frames = torch.empty((nframes, lat.n), dtype=torch.int8, device="cuda")
    lat.init()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.advance_frames(T, frame_dt, frames, 1)
    torch.cuda.synchronize()
    dt_f = time.perf_counter() - t0
    lat.close()
    base = rows[0]["ms"] if rows and rows[0]["lag"] is None else None
    return {"workload": "square_4096", "T": T, "rows": rows,
            "frames": {"dt": frame_dt, "count": nframes, "ms": dt_f * 1e3,
                       "ms_without": base}}


def bench_range(qs=(1, 2, 3), steps: int = 3, cpu_sample_T: float = 0.5) -> dict:
    """q-th degree neighbourhoods on a 1024^2 torus to T = 50: spin-updates per
    second per reach, each run checked against the one-shot result of another
    tiling, and the oracle on one host core for reach 2 (bounded sample)."""
    import torch
    from paper_cs_0502039_amd import aca, workloads
    rows = []
    for q in qs:
        params = workloads.square_1024_range(q) if q > 1 else dict(
            workloads.square_1024_range(2), range=1, beta=0.4)
        lat = aca.Lattice(params)
        lat.init().advance(params["T"])
        ref = lat.read()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            lat.init().advance(params["T"])
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        st = lat.stats()
        other = aca.Lattice(params, tuning=dict(tile=(40, 40), ghost=(2, 2), max_sweeps=20))
        other.init().advance(params["T"])
        same = all(np.array_equal(x, y) for x, y in zip(ref, other.read()))
        other.close()
        rows.append({"range": q, "neighbours": len(aca.thresholds(params)) // 2 - 1,
                     "beta": params["beta"], "ms": dt * 1e3,
                     "spin_updates_per_s": st["events"] / dt, "launches": st["launches"],
                     "tuning": lat.tuning(), "tilings_agree": same})
        log(f"range {q}: {dt * 1e3:.1f} ms, {st['events'] / dt:.3e} spin-updates/s")
        lat.close()
    out = {"workload": "square_1024_range", "T": 50.0, "rows": rows}
    if cpu_sample_T > 0:
        import oracle
        params = workloads.square_1024_range(2)
        s, t, n = oracle.init(params)
        t0 = time.time()
        ev, _ = oracle.run(params, cpu_sample_T, s, t, n)
        out["cpu_baseline"] = {"value": ev / (time.time() - t0), "unit": "spin-updates/s",
                               "cores": 1, "kind": "oracle",
                               "sample": f"1024^2, range 2, initial state to T={cpu_sample_T}"}
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="square_4096")
    ap.add_argument("--cpu-sample-T", type=float, default=1.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--tile", type=int, nargs="*", default=None)
    ap.add_argument("--ghost", type=int, nargs="*", default=None)
    ap.add_argument("--sweeps", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a 2 GiB device copy (for counter scaling)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the automatic schedules instead of tuning on the workload")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--only", choices=("single", "batched", "served", "lag", "range"),
                    default=None)
    ap.add_argument("--serve-jobs", type=int, default=400)
    ap.add_argument("--serve-arena-gib", type=float, default=64.0)
    ap.add_argument("--serve-slots", type=int, default=512)
    # device time per server step: longer steps spread the per-step host work
    # (admission, pack/unpack, the counter read-back) over more epochs; the
    # step length also bounds how long a finished job waits to be reported
    ap.add_argument("--serve-budget-ms", type=float, default=16.0)
    ap.add_argument("--no-cpu-aggregate", action="store_true")
    ap.add_argument("--cpu-aggregate-only", type=int, default=0, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_aggregate_only:
        cpu_aggregate_main(args.cpu_aggregate_only)
        return 0
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: runs on one GPU only; the workload is a single lattice on "
              "one device, and runs over several GPUs are not supported.", file=sys.stderr)
        return 2

    # the all-core oracle runs in a child interpreter, started before this
    # process touches the GPU
    aggregate = None
    if args.only is None and not (args.no_cpu_baseline or args.no_cpu_aggregate):
        aggregate = cpu_aggregate()

    import torch
    from paper_cs_0502039_amd import aca, workloads

    torch.cuda.set_device(0)
    if args.only == "batched":
        print(json.dumps({"batched": bench_batched(args.steps, args.warmup,
                                                   not args.no_autotune)}), flush=True)
        return 0
    if args.only == "lag":
        print(json.dumps({"lag": bench_lag([0.0, 16.0, 8.0, 4.0, 2.0, 1.0, 0.5, 0.3])}),
              flush=True)
        return 0
    if args.only == "range":
        print(json.dumps({"range": bench_range()}), flush=True)
        return 0
    if args.only == "served":
        print(json.dumps({"served": bench_served(args.serve_arena_gib, args.serve_slots,
                                                 args.serve_budget_ms, args.serve_jobs)}),
              flush=True)
        return 0

    params = getattr(workloads, args.workload)()
    T = params["T"]
    if args.calibrate_copy:
        copy_calibration()
    lat = aca.Lattice(params)
    if args.tile or args.ghost or args.sweeps or args.block:
        kw = {}
        if args.tile:
            kw["tile"] = tuple(args.tile)
        if args.ghost:
            kw["ghost"] = tuple(args.ghost)
        if args.sweeps:
            kw["max_sweeps"] = args.sweeps
        if args.block:
            kw["block"] = args.block
        lat.set_tuning(**kw)
    tune = None
    if not (args.no_autotune or args.tile or args.ghost or args.sweeps or args.block):
        # the tuner advances the real lattice slice by slice; the warm-up pass
        # then finishes it (same final state whichever schedule wins)
        lat.init()
        # a slice should span several launches: a slice's last launch is a
        # partial one that costs nearly a whole launch, which would favour
        # the candidates with fewer rounds per visit in short slices.  On a
        # large 2D lattice five strong candidates of T/6 each leave a sixth of
        # the horizon for the finish; elsewhere the library's set, T/20 each
        cands = None
        if params["dim"] == 2 and min(params["L"]) >= 1024:
            cands = [dict(tile=(72, 54), ghost=(5, 5), max_sweeps=40),
                     dict(tile=(64, 60), ghost=(5, 5), max_sweeps=40),
                     dict(tile=(72, 54), ghost=(5, 5), max_sweeps=32),
                     dict(tile=(64, 60), ghost=(5, 5), max_sweeps=32),
                     dict(tile=(64, 52), ghost=(5, 5), max_sweeps=32)]
        tune = lat.tune(max(T / (6.0 if cands else 20.0), 1e-3), cands)
        lat.advance(T)
        log(f"autotuned: {tune['tuning']} (rates per ms "
            f"{[round(r) for r in tune['rates_per_ms']]})")
    log(f"bench: {args.workload} L={params['L']} T={T} tuning={lat.tuning()}")

    for i in range(args.warmup):
        lat.init().advance(T)
        log(f"warmup {i}: {lat.stats()['device_ms']:.1f} ms")
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        lat.init().advance(T)
        stats.append(lat.stats())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    for i, st in enumerate(stats):
        log(f"step {i}: {st['device_ms']:.1f} ms, {st['launches']} launches, "
            f"kernel {st['kernel_ms']:.1f} ms")

    st = stats[-1]
    events = st["events"]
    # Section 4's efficiency counters cost the visit a few per cent, so the
    # timed steps run without them; one more advance, untimed, collects them
    lat.set_counting(True)
    lat.init().advance(T)
    st_eff = lat.stats()
    trace = lat.trace()
    lat.set_counting(False)
    ms_per_step = 1e3 * elapsed / args.steps
    value = events / (elapsed / args.steps)

    # roofline of the visit kernel, per launch
    launches = st["launches"]
    t_launch = st["kernel_ms"] / 1e3 / launches
    bytes_launch = st["region_bytes"] / launches
    hbm_achieved = bytes_launch / t_launch / 1e9
    ev_launch = events / launches
    alu_achieved = ev_launch / t_launch / 1e9                  # Gevents/s
    alu_peak = VALU_LANE_OPS_PER_S / SLOTS_PER_EVENT / 1e9      # Gevents/s
    traffic = measured_traffic(args.workload, lat.tuning())
    hbm = {"bound": "hbm", "achieved": hbm_achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": hbm_achieved / HBM_PEAK_GBS, "traffic": traffic}
    alu = {"bound": "alu", "achieved": alu_achieved, "peak": alu_peak,
           "unit": "Garrivals/s", "frac": alu_achieved / alu_peak, "traffic": traffic}
    roofline = alu if alu["frac"] >= hbm["frac"] else hbm
    other = hbm if roofline is alu else alu

    bit_exact = None
    if not args.no_check:
        gold_path = os.path.join(ROOT, "tests", "golden", f"{args.workload}.json")
        if os.path.exists(gold_path):
            with open(gold_path) as f:
                gold = json.load(f)
            s, t, n = lat.read()
            bit_exact = digest(s, t, n) == (gold["sha256_s"], gold["sha256_t"],
                                            gold["sha256_n"]) and gold["events"] == events
            log(f"bit-exact vs oracle digest: {bit_exact}")

    out = {
        "metric": "spin-updates/s at 4096^2 (bit-exact); batched vs plain speedup; "
                  "p99 job latency",
        "value": value,
        "unit": "spin-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "dim": params["dim"], "L": params["L"],
                   "T": T, "beta": params["beta"], "h": params["h"], "rule": params["rule"],
                   "init": params["init"], "seed": params["seed"],
                   "tuning": lat.tuning(), "autotuned": tune is not None},
        "roofline": roofline,
        "roofline_other": other,
        "bit_exact": bit_exact,
        "events": events,
        "flips": st["flips"],
        "launches": launches,
        "kernel_ms_per_launch": t_launch * 1e3,
        "sweeps_per_visit": st["sweeps"] / st["visits"],
        "enabled_per_check": (events + st["ghost_events"]) / max(1, st["cell_checks"]),
        "ghost_events_per_event": st["ghost_events"] / max(1, events),
        # Section 4's efficiency N0 / N: the fraction of cells that pass the
        # enabling test at an iteration.  first_scan: the first launch's scan
        # of the initial state (the first synchronous iteration, expected
        # 1/(z+1)); scan: every launch's initial scan over the owned cells
        # before the horizon; per_round: arrivals applied per simulated cell
        # per worklist round inside the regions.  The paper's long-run 2D
        # value of the synchronous iteration is 0.121.
        "efficiency": {
            "first_scan": trace[0]["scan_enabled"] / max(1, trace[0]["scan_live"]),
            "scan": st_eff["scan_enabled"] / max(1, st_eff["scan_live"]),
            "per_round": (st_eff["events"] + st_eff["ghost_events"])
            / max(1, st_eff["round_cells"]),
            "paper_2d_long_run": 0.121},
        # what a captured graph of the launch loop could save at most: the
        # advance's wall time less its kernels' time
        "launch_gap_ms_per_step": st["device_ms"] - st["kernel_ms"],
    }
    lat.close()
    del lat
    if args.only is None:
        out["other_configs"] = {n: bench_config(n) for n in ("square_64", "cubic_256")
                                if n != args.workload}
    if args.only is None and not args.no_batched:
        out["batched"] = bench_batched(args.steps, args.warmup, not args.no_autotune)
    if args.only is None and not args.no_served:
        out["served"] = bench_served(args.serve_arena_gib, args.serve_slots,
                                     args.serve_budget_ms, args.serve_jobs)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(params, args.cpu_sample_T)
        if aggregate is not None:
            out["cpu_baseline"]["all_cores_batch_512"] = aggregate
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
