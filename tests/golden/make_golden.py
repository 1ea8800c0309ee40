"""Write the oracle's expected results for the full-size workloads.

Calls only the oracle (``oracle.simulate``); nothing here touches the GPU library.
For each named workload it stores, in ``tests/golden/<name>.json``, SHA-256
digests of the final spins (int8), times (float64, little endian) and counts
(uint32, little endian), plus totals useful for diagnosis.

Usage:  python tests/golden/make_golden.py square_64 square_4096 cubic_256
        python tests/golden/make_golden.py batch_512 --jobs 6
        python tests/golden/make_golden.py served_16 --jobs 5

``served_16`` holds the first 16 jobs of the served stream at full size (the
same parameters the serving benchmark submits first), one entry per job id.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_cs_0502039_amd import workloads  # noqa: E402


def digest_state(s, t, n) -> dict:
    return {
        "sha256_s": hashlib.sha256(s.tobytes()).hexdigest(),
        "sha256_t": hashlib.sha256(t.astype("<f8").tobytes()).hexdigest(),
        "sha256_n": hashlib.sha256(n.astype("<u4").tobytes()).hexdigest(),
        "sum_s": int(s.astype("int64").sum()),
        "sum_n": int(n.astype("int64").sum()),
        "min_t": float(t.min()),
    }


def solve(params: dict) -> dict:
    t0 = time.time()
    s, t, n, ev, fl = oracle.simulate(params, params["T"])
    out = {"params": params, "events": ev, "flips": fl,
           "oracle_seconds": round(time.time() - t0, 2)}
    out.update(digest_state(s, t, n))
    return out


def _solve_batch_item(args):
    i, params = args
    return i, solve(params)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="+")
    ap.add_argument("--jobs", type=int, default=1)
    a = ap.parse_args()
    oracle.lib()
    for name in a.names:
        path = os.path.join(HERE, f"{name}.json")
        if name in ("batch_512", "served_16"):
            from multiprocessing import Pool
            if name == "batch_512":
                items = list(enumerate(workloads.batch_512()))
            else:
                items = [(j["id"], {k: v for k, v in j.items() if k not in ("t_arrive", "id")})
                         for j in workloads.served_stream()[:16]]
            results = [None] * len(items)
            # largest first, so the pool drains evenly
            order = sorted(items, key=lambda it: -it[1]["L"][0] ** it[1]["dim"] * it[1]["T"])
            with Pool(a.jobs) as pool:
                for i, res in pool.imap_unordered(_solve_batch_item, order):
                    results[i] = res
                    print(f"{name} item {i} done ({res['oracle_seconds']} s)", flush=True)
            doc = {"workload": name, "items": results}
        else:
            params = getattr(workloads, name)()
            doc = {"workload": name, **solve(params)}
        with open(path + ".tmp", "w") as f:
            json.dump(doc, f, indent=1)
        os.replace(path + ".tmp", path)
        print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    main()
