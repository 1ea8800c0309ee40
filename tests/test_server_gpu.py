"""GPU tests of the job server (continuous batching, through the C-ABI).

Each served job must end bit-identical to the same job run alone (init +
advance on its own) and to the serial oracle, whatever jobs it shared the GPU
with, when it was admitted, and how the arena budget delayed it: the trajectory
of a lattice is unique (argument after Fig. 3.1), so the tolerance is zero.
"""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

import oracle
from paper_cs_0502039_amd import aca, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a visible GPU"
    aca.load()
    return t


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def assert_same_state(a, b, label=""):
    s1, t1, n1 = a
    s2, t2, n2 = b
    assert s1.shape == s2.shape, label
    bad_s = np.flatnonzero(s1 != s2)
    bad_t = np.flatnonzero(t1.view(np.uint64) != t2.view(np.uint64))
    bad_n = np.flatnonzero(n1 != n2)
    assert bad_s.size == 0 and bad_t.size == 0 and bad_n.size == 0, (
        f"{label}: {bad_s.size} spins, {bad_t.size} times, {bad_n.size} counts differ")


def small_stream(count=36):
    """Jobs with the served mix's shape (2D and 3D, both rules, uneven sizes and
    horizons) scaled down so the oracle checks every one in seconds."""
    rng = np.random.default_rng(55)
    jobs = []
    for j in range(count):
        if rng.uniform() < 0.8:
            side = int(np.rint(np.exp(rng.uniform(np.log(12), np.log(120)))))
            dims, L = 2, (side, side)
        else:
            side = int(rng.integers(6, 24))
            dims, L = 3, (side, side, side)
        rule = "glauber" if rng.uniform() < 0.5 else "metropolis"
        jobs.append(workloads.lattice(dims, L, float(rng.uniform(0.15, 0.6)), rule,
                                      seed=10**6 + j, T=float(rng.uniform(1.0, 12.0))))
    return jobs


def drive(server, jobs, per_step=3, budget_ms=0.2):
    """Submit jobs a few per step (arrivals while others run), step until all
    are done; returns {job index: (state, stats)} read right after finishing."""
    ids = {}
    results = {}
    pending = list(range(len(jobs)))
    steps = 0
    while pending or len(results) < len(jobs):
        for _ in range(per_step):
            if pending:
                i = pending.pop(0)
                ids[server.submit(jobs[i])] = i
        for job in server.step(budget_ms):
            state, st = server.job(job)
            assert state == aca.JOB_DONE
            results[ids[job]] = (server.read(job), st)
            server.release(job)
        steps += 1
        assert steps < 100000
    return results


def test_served_jobs_equal_alone_and_oracle(torch):
    jobs = small_stream()
    big = max(aca.job_bytes(p) for p in jobs)
    server = aca.Server(arena_bytes=4 * big, max_jobs=8)   # admission waits on memory
    say(f"serving {len(jobs)} jobs, arena {4 * big} bytes")
    results = drive(server, jobs)
    st = server.stats()
    assert st["finished"] == len(jobs) and st["failed"] == 0
    assert st["arena_peak"] <= st["arena_bytes"]
    assert st["queued_peak"] > 0
    for i, p in enumerate(jobs):
        (s, t, n), jst = results[i]
        s1, t1, n1, st1 = aca.simulate(p)
        assert_same_state((s, t, n), (s1, t1, n1), f"job {i} alone vs mix")
        so, to, no, ev, fl = oracle.simulate(p, p["T"])
        assert_same_state((s, t, n), (so, to, no), f"job {i} vs oracle")
        assert jst["events"] == ev and jst["flips"] == fl
        assert jst["last_T"] == p["T"]
    server.close()


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "served_16.json")


def digest(s, t, n):
    return (hashlib.sha256(s.tobytes()).hexdigest(),
            hashlib.sha256(t.astype("<f8").tobytes()).hexdigest(),
            hashlib.sha256(n.astype("<u4").tobytes()).hexdigest())


def test_served_stream_jobs_alone_vs_mix(torch):
    """The first 16 jobs of the served workload at full size (2D tori up to
    1572^2 and 3D cubes up to 74^3, both rules, horizons up to 992; 4.9e9
    arrivals), served together with a small step budget, equal the oracle's
    digests (tests/golden/served_16.json, written by make_golden.py from the
    oracle alone) and each job run alone; sampled cell clocks equal the
    oracle's closed form."""
    with open(GOLDEN) as f:
        gold = json.load(f)["items"]
    jobs = [dict(j) for j in workloads.served_stream(count=len(gold))]
    for j in jobs:
        j.pop("t_arrive")
        j.pop("id")
    for g, p in zip(gold, jobs):
        assert g["params"] == p, "golden file is for other job parameters"
    server = aca.Server(arena_bytes=sum(aca.job_bytes(p) for p in jobs), max_jobs=16)
    say("serving the first served-stream jobs")
    results = drive(server, jobs, per_step=2, budget_ms=2.0)
    rng = np.random.default_rng(3)
    for i, p in enumerate(jobs):
        (s, t, n), jst = results[i]
        say(f"stream job {i}: {p['dim']}D side {p['L'][0]} T={p['T']:.1f}")
        assert digest(s, t, n) == (gold[i]["sha256_s"], gold[i]["sha256_t"],
                                   gold[i]["sha256_n"]), f"stream job {i} vs oracle digest"
        assert jst["events"] == gold[i]["events"] and jst["flips"] == gold[i]["flips"]
        s1, t1, n1, st1 = aca.simulate(p)
        assert_same_state((s, t, n), (s1, t1, n1), f"stream job {i}")
        assert jst["events"] == st1["events"] == int(n.astype(np.int64).sum())
        cells = rng.choice(s.size, size=256, replace=False).astype(np.uint32)
        tc, nc = oracle.cell_clock(p, cells, p["T"])
        assert np.array_equal(t[cells].view(np.uint64), tc.view(np.uint64))
        assert np.array_equal(n[cells], nc)
    server.close()


def test_server_budget_limits_concurrency(torch):
    jobs = [workloads.lattice(2, (64, 64), 0.4, seed=40 + i, T=6.0) for i in range(6)]
    one = aca.job_bytes(jobs[0])
    server = aca.Server(arena_bytes=2 * one + 100, max_jobs=8)
    for p in jobs:
        server.submit(p)
    seen_running = 0
    done = set()
    while len(done) < len(jobs):
        for job in server.step(0.05):
            done.add(job)
            server.release(job)             # frees arena room for the next one
        q, r = server.load()
        seen_running = max(seen_running, r)
    assert seen_running <= 2
    st = server.stats()
    assert st["arena_peak"] <= 2 * one
    assert st["queued_peak"] == len(jobs)
    server.close()


def test_server_state_errors(torch):
    p = workloads.lattice(2, (48, 48), 0.3, T=4.0)
    server = aca.Server(arena_bytes=2 * aca.job_bytes(p), max_jobs=2)
    with pytest.raises(aca.AcaError) as e:
        server.submit(workloads.lattice(2, (512, 512), 0.3, T=1.0))   # never fits
    assert e.value.code == aca.ACA_ENOMEM
    with pytest.raises(aca.AcaError) as e:
        server.submit(workloads.lattice(2, (48, 48), 0.3, T=2.0 ** 31))  # rate * T > 2^30
    assert e.value.code == aca.ACA_EINVAL
    job = server.submit(p)
    with pytest.raises(aca.AcaError) as e:
        server.read(job)                     # queued
    assert e.value.code == aca.ACA_ESTATE
    with pytest.raises(aca.AcaError) as e:
        server.release(job)
    assert e.value.code == aca.ACA_ESTATE
    with pytest.raises(aca.AcaError) as e:
        server.close()                       # queued work
    assert e.value.code == aca.ACA_ESTATE
    done = []
    while not done:
        done = server.step(0.0)
    assert done == [job]
    s, t, n = server.read(job)
    so, to, no, _, _ = oracle.simulate(p, p["T"])
    assert_same_state((s, t, n), (so, to, no), "single served job")
    server.release(job)
    with pytest.raises(aca.AcaError) as e:
        server.job(job)                      # forgotten
    assert e.value.code == aca.ACA_EINVAL
    server.close()
