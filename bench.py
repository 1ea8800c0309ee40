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
  cpu_baseline  the serial oracle timed on a bounded sample of the same workload
                on one host core.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Plain VALU issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one wave64
# instruction every 4 cycles per SIMD; binary64 add/mul run at this rate).
VALU_LANE_OPS_PER_S = 256 * 4 * 16 * 2.4e9
# Issue slots one applied arrival needs at minimum on gfx950: Philox4x32-10 is
# 20 v_mad_u64_u32 (half rate, 2 slots each) and 20 v_bitop3_b32; -ln u is 51
# binary64 slots (16 mul, 16 add, the division sequence with its quarter-rate
# reciprocal, conversions) and 11 integer ones; flip test and clock update 8.
SLOTS_PER_EVENT = 40 + 20 + 51 + 11 + 8


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def digest(s, t, n):
    return (hashlib.sha256(s.tobytes()).hexdigest(),
            hashlib.sha256(t.astype("<f8").tobytes()).hexdigest(),
            hashlib.sha256(n.astype("<u4").tobytes()).hexdigest())


VISIT_SOURCES = ("aca_device.h", "aca_internal.h", "aca_visit_fast.hip")


def kernel_source_digest() -> str:
    """SHA-256 over the sources the tile-visit kernel of the large lattices is
    compiled from."""
    csrc = os.path.join(ROOT, "paper_cs_0502039_amd", "csrc")
    h = hashlib.sha256()
    for name in VISIT_SOURCES:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic(workload: str, launches: int):
    """HBM bytes per visit launch from the committed counter summary
    (profiles/traffic_<workload>.json, FETCH_SIZE + WRITE_SIZE scaled by a copy
    kernel's readings), or None when it is missing or the kernels changed since."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        doc = json.load(f)
    if doc.get("kernel_source_sha256") != kernel_source_digest():
        return None
    return doc["hbm_bytes_per_launch"]


def copy_calibration(nbytes: int = 1 << 31) -> None:
    """A plain device copy of known size, for scaling FETCH_SIZE / WRITE_SIZE."""
    import torch
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    log(f"copy calibration: {nbytes} bytes read and {nbytes} bytes written")


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
            "sample": (f"{params['L'][0]}^{params['dim']} lattice seed {params['seed']}, "
                       f"binary-heap oracle from the initial state to T={T_sample} "
                       f"({ev} arrivals in {t2 - t1:.1f} s; init {t1 - t0:.1f} s not "
                       f"counted)")}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="square_4096")
    ap.add_argument("--cpu-sample-T", type=float, default=0.5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--tile", type=int, nargs="*", default=None)
    ap.add_argument("--ghost", type=int, nargs="*", default=None)
    ap.add_argument("--sweeps", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a 2 GiB device copy (for counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only; the workload is a single "
              "lattice per GPU and multi-GPU runs are not part of it (see DESIGN.md, "
              "sharding).", file=sys.stderr)
        return 2

    import torch
    from paper_cs_0502039_amd import aca, workloads

    params = getattr(workloads, args.workload)()
    T = params["T"]
    torch.cuda.set_device(0)
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
    traffic = measured_traffic(args.workload, launches)
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
        "metric": "spin-updates/s at 4096^2 (bit-exact)",
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
                   "tuning": lat.tuning()},
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
    }
    lat.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(params, args.cpu_sample_T)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
