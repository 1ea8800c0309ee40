"""GPU parity of the persistent batch kernel (through the C-ABI).

Every member of a batch must end bit-identical to the serial oracle run of that
lattice alone -- whatever the mix it shares the GPU with, the order it joins in,
the step budget and the tiling -- because the trajectory is unique (argument after
Fig. 3.1) and the aggregation is partition-invariant (Fig. 3.4).
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
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


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
        f"{label}: {bad_s.size} spins, {bad_t.size} times, {bad_n.size} counts differ; "
        f"first cells {bad_s[:5]}, {bad_t[:5]}, {bad_n[:5]}")


def oracle_state(p, T=None):
    s, t, n, ev, fl = oracle.simulate(p, p["T"] if T is None else T)
    return (s, t, n), ev, fl


def mixed_cases():
    """Small lattices of every dimension, both rules, ragged sides, side 2,
    different horizons; cheap enough for the oracle."""
    cases = workloads.small_cases()
    rng = np.random.default_rng(21)
    for i in range(10):
        side = int(rng.integers(8, 90))
        cases.append(workloads.lattice(2, (side, int(rng.integers(8, 90))),
                                       float(rng.uniform(0.2, 0.6)),
                                       "glauber" if i % 2 else "metropolis",
                                       seed=700 + i, T=float(rng.uniform(2, 25))))
    for i in range(3):
        side = int(rng.integers(5, 20))
        cases.append(workloads.lattice(3, (side, side + 1, side + 2),
                                       float(rng.uniform(0.1, 0.4)), "metropolis",
                                       h=0.2, seed=800 + i, T=float(rng.uniform(2, 10))))
    return cases


@pytest.fixture(scope="module")
def mixed_expected():
    cases = mixed_cases()
    return cases, [oracle_state(p) for p in cases]


def run_batch(cases, capacity=None, tuning=None, T=None):
    lats = [aca.Lattice(p).init() for p in cases]
    batch = aca.Batch(capacity or len(cases))
    for dim, kw in (tuning or {}).items():
        batch.set_tuning(dim, **kw)
    batch.advance(lats, [p["T"] for p in cases] if T is None else T)
    out = [l.read() for l in lats]
    stats = [l.stats() for l in lats]
    bstats = batch.stats()
    batch.close()
    for l in lats:
        l.close()
    return out, stats, bstats


def test_mixed_batch_matches_oracle(torch, mixed_expected):
    cases, expected = mixed_expected
    say(f"batch of {len(cases)} mixed lattices")
    got, stats, bstats = run_batch(cases)
    assert bstats["finished"] == len(cases)
    for p, g, (want, ev, fl), st in zip(cases, got, expected, stats):
        label = f"{p['dim']}D L={p['L']} T={p['T']:.3f} seed={p['seed']}"
        assert_same_state(g, want, label)
        assert st["events"] == ev, label
        assert st["flips"] == fl, label
        assert st["last_T"] == p["T"]


@pytest.mark.parametrize("tuning", [
    {2: dict(tile=(8, 8), ghost=(1, 1), max_sweeps=1), 3: dict(tile=(4, 4, 4), ghost=(0, 0, 0),
                                                              max_sweeps=2),
     1: dict(tile=(64,), ghost=(3,), max_sweeps=3)},
    {2: dict(tile=(32, 16), ghost=(6, 2), max_sweeps=1000), 3: dict(tile=(8, 4, 6),
                                                                    ghost=(2, 1, 3))},
], ids=["small-tiles", "odd-tiles"])
def test_batch_tiling_does_not_change_results(torch, mixed_expected, tuning):
    cases, expected = mixed_expected
    say(f"batch tiling {tuning}")
    got, _, _ = run_batch(cases, tuning=tuning)
    for p, g, (want, _, _) in zip(cases, got, expected):
        assert_same_state(g, want, f"{p['dim']}D L={p['L']} seed={p['seed']}")


def test_stepwise_batch_with_late_joiners(torch, mixed_expected):
    """Continuous batching: members join between steps of one epoch each and
    leave as they finish; results equal the oracle's."""
    cases, expected = mixed_expected
    say("stepwise batch with joiners")
    lats = [aca.Lattice(p).init() for p in cases]
    batch = aca.Batch(8)            # fewer slots than lattices: admit as they free up
    waiting = list(range(len(cases)))
    done_order = []
    steps = 0
    while waiting or batch._members:
        while waiting and len(batch._members) < batch.capacity:
            i = waiting.pop(0)
            batch.attach(lats[i], cases[i]["T"])
        batch.step(budget_ms=0.0, max_epochs=1 + steps % 3)
        steps += 1
        for lat in batch.poll():
            done_order.append(lats.index(lat))
        assert steps < 100000
    assert sorted(done_order) == list(range(len(cases)))
    for i, (p, (want, ev, fl)) in enumerate(zip(cases, expected)):
        assert_same_state(lats[i].read(), want, f"case {i}")
        assert lats[i].stats()["events"] == ev
    batch.close()
    for l in lats:
        l.close()


def test_batch_time_budget_and_chunks(torch, mixed_expected):
    """A tiny device-time budget per step pauses members at epoch boundaries;
    advancing in two chunks of horizon gives the one-shot result."""
    cases, expected = mixed_expected
    lats = [aca.Lattice(p).init() for p in cases]
    batch = aca.Batch(len(cases))
    for lat, p in zip(lats, cases):
        batch.attach(lat, p["T"] / 3)
    while batch.step(budget_ms=0.05) > 0:
        pass
    assert len(batch.poll()) == len(cases)
    batch.advance(lats, [p["T"] for p in cases])
    assert batch.stats()["steps"] > 2
    for i, (p, (want, _, _)) in enumerate(zip(cases, expected)):
        assert_same_state(lats[i].read(), want, f"case {i}")
    batch.close()
    for l in lats:
        l.close()


def test_batch_equals_single_lattice_path(torch):
    """Medium lattices: batch result equals aca_advance alone (both GPU), and a
    sample of cells' clocks equals the oracle's closed-form clocks."""
    rng = np.random.default_rng(33)
    cases = []
    for i in range(12):
        side = int(np.rint(np.exp(rng.uniform(np.log(40), np.log(400)))))
        cases.append(workloads.lattice(2, (side, side), float(rng.uniform(0.2, 0.6)),
                                       seed=900 + i, T=float(rng.uniform(5, 40))))
    cases.append(workloads.lattice(3, (48, 40, 36), 0.22, "metropolis", h=0.1, seed=950, T=12.0))
    got, _, _ = run_batch(cases)
    for p, g in zip(cases, got):
        s, t, n, _ = aca.simulate(p)
        assert_same_state(g, (s, t, n), f"L={p['L']}")
        cells = rng.choice(s.size, size=min(s.size, 3000), replace=False).astype(np.uint32)
        tc, nc = oracle.cell_clock(p, cells, p["T"])
        assert np.array_equal(g[1][cells].view(np.uint64), tc.view(np.uint64))
        assert np.array_equal(g[2][cells], nc)


def test_batch_takes_long_1d_lattices(torch):
    """1D members whose tiles are thousands of cells long (a line cut into two
    tiles of about 8000) fit a region's LDS and match the oracle, next to 2D
    and 3D members."""
    cases = [workloads.lattice(1, (16264,), 0.45, seed=16, T=15.0),
             workloads.lattice(1, (20000,), 0.4, "metropolis", h=0.1, seed=19, T=12.0,
                               rate=0.37),
             workloads.lattice(2, (40, 33), 0.4, seed=17, T=10.0),
             workloads.lattice(3, (12, 10, 9), 0.2, "metropolis", seed=20, T=6.0)]
    say("batch with long 1D lattices")
    got, stats, bstats = run_batch(cases)
    assert bstats["finished"] == len(cases)
    for p, g, st in zip(cases, got, stats):
        want, ev, fl = oracle_state(p)
        assert_same_state(g, want, f"{p['dim']}D L={p['L']}")
        assert st["events"] == ev and st["flips"] == fl


def test_batch_state_errors(torch):
    p = workloads.lattice(2, (16, 16), 0.3, T=3.0)
    lat = aca.Lattice(p).init()
    other = aca.Lattice(p)           # never initialised
    batch = aca.Batch(1)
    with pytest.raises(aca.AcaError) as e:
        batch.attach(other, 1.0)
    assert e.value.code == aca.ACA_ESTATE
    with pytest.raises(aca.AcaError) as e:
        batch.attach(lat, 2.0 ** 31)  # rate * T > 2^30
    assert e.value.code == aca.ACA_EINVAL
    batch.attach(lat, 2.0)
    with pytest.raises(aca.AcaError) as e:
        batch.attach(lat, 2.0)
    assert e.value.code == aca.ACA_ESTATE
    for call in (lambda: lat.advance(3.0), lambda: lat.read(), lambda: lat.init(),
                 lambda: lat.set_tuning(max_sweeps=3), lambda: lat.resume(1.0)):
        with pytest.raises(aca.AcaError) as e:
            call()
        assert e.value.code == aca.ACA_ESTATE
    assert lat.lib.aca_destroy(lat._h) == aca.ACA_ESTATE
    other.init()
    with pytest.raises(aca.AcaError) as e:
        batch.attach(other, 1.0)      # full
    assert e.value.code == aca.ACA_ENOMEM
    with pytest.raises(aca.AcaError) as e:
        batch.close()                 # still has a member
    assert e.value.code == aca.ACA_ESTATE
    while batch.step() > 0:
        pass
    assert batch.poll() == [lat]
    with pytest.raises(aca.AcaError) as e:
        batch.attach(lat, 1.0)        # before its last horizon
    assert e.value.code == aca.ACA_EINVAL
    want, _, _ = oracle_state(p, 2.0)
    assert_same_state(lat.read(), want, "after batch")
    lat.advance(3.0)                  # detached: the single path continues
    want, _, _ = oracle_state(p, 3.0)
    assert_same_state(lat.read(), want, "after single advance")
    batch.close()
    lat.close()
    other.close()


# ------------------------------------------------------------ full-size batch

def digest(s, t, n):
    return (hashlib.sha256(s.tobytes()).hexdigest(),
            hashlib.sha256(t.astype("<f8").tobytes()).hexdigest(),
            hashlib.sha256(n.astype("<u4").tobytes()).hexdigest())


def test_batch_512_full_size(torch):
    """The 512-lattice workload in one batch: every lattice's sampled cell clocks
    equal the oracle's; when the oracle's digests are present, every final state
    equals the oracle's exactly."""
    cases = workloads.batch_512()
    gold = None
    path = os.path.join(GOLDEN, "batch_512.json")
    if os.path.exists(path):
        with open(path) as f:
            gold = json.load(f)["items"]
    say("batch_512 full size")
    lats = [aca.Lattice(p).init() for p in cases]
    batch = aca.Batch(len(cases))
    batch.advance(lats, [p["T"] for p in cases])
    st = batch.stats()
    say(f"batch_512: {st['events']} arrivals, {st['kernel_ms']:.0f} ms kernel, "
        f"{st['steps']} steps")
    rng = np.random.default_rng(17)
    total = 0
    for i, (p, lat) in enumerate(zip(cases, lats)):
        s, t, n = lat.read()
        cells = rng.choice(s.size, size=64, replace=False).astype(np.uint32)
        tc, nc = oracle.cell_clock(p, cells, p["T"])
        assert np.array_equal(t[cells].view(np.uint64), tc.view(np.uint64)), i
        assert np.array_equal(n[cells], nc), i
        total += int(n.astype(np.int64).sum())
        if gold is not None:
            assert gold[i]["params"] == p
            assert digest(s, t, n) == (gold[i]["sha256_s"], gold[i]["sha256_t"],
                                       gold[i]["sha256_n"]), i
            assert lat.stats()["flips"] == gold[i]["flips"], i
        lat.close()
    assert total == st["events"]
    batch.close()


def test_batch_autotune_keeps_results(torch, mixed_expected):
    """The batch tuner advances the real lattices slice by slice under each
    candidate; finishing afterwards gives the oracle's result."""
    cases, expected = mixed_expected
    lats = [aca.Lattice(p).init() for p in cases]
    batch = aca.Batch(len(cases))
    cands = [dict(tile=(16, 16), ghost=(2, 2), max_sweeps=8),
             dict(tile=(8, 24), ghost=(1, 3), max_sweeps=3),
             dict(tile=(64, 56), ghost=(4, 4), max_sweeps=32)]
    res = batch.tune(lats, [p["T"] for p in cases], 2, cands, frac=0.1)
    assert 0 <= res["best"] < len(cands)
    assert len(res["rates_per_ms"]) == len(cands) and min(res["rates_per_ms"]) > 0
    want_tile = list(cands[res["best"]]["tile"]) + [0]
    assert res["tuning"]["tile"] == want_tile
    res3 = batch.tune(lats, [p["T"] for p in cases], 3, None, frac=0.05)   # library set
    assert len(res3["rates_per_ms"]) >= 4
    batch.advance(lats, [p["T"] for p in cases])
    for i, (p, (want, ev, fl)) in enumerate(zip(cases, expected)):
        assert_same_state(lats[i].read(), want, f"case {i}")
        assert lats[i].stats()["events"] == ev
    batch.close()
    for l in lats:
        l.close()
