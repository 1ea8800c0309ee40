"""Randomized GPU parity against the serial oracle, bit for bit.

Seeded draws over everything a caller may vary: dimension, sides (down to
2, odd, ragged against the tile), rule, coupling and field signs and sizes,
temperature, rate, initial state, horizon, and the schedule (tile, ghost
width, rounds per visit, workgroup size).  By the uniqueness of the
trajectory (the argument after Fig. 3.1) and the partition invariance of
aggregated cells (Fig. 3.4), every draw must give the oracle's spins, times
and counts exactly; a schedule whose region does not fit a workgroup's LDS
must be refused, not run.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_cs_0502039_amd import aca, workloads

pytestmark = pytest.mark.gpu

N_DRAWS = 48


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a visible GPU"
    aca.load()
    return t


def draw(i):
    rng = np.random.default_rng(9000 + i)
    dim = int(rng.integers(1, 4))
    hi = {1: 3000, 2: 90, 3: 26}[dim]
    L = [int(rng.choice([2, 3, int(rng.integers(2, hi + 1))])) if rng.uniform() < 0.15
         else int(rng.integers(4, hi + 1)) for _ in range(dim)]
    n = int(np.prod(L))
    rule = "glauber" if rng.uniform() < 0.5 else "metropolis"
    J = float(rng.choice([1.0, -1.0, 0.5, 0.0]))
    h = float(rng.choice([0.0, 0.0, 0.2, -0.35]))
    beta = float(rng.uniform(0.0, 1.0))
    init = str(rng.choice(["random", "random", "plus", "minus"]))
    rate = float(rng.choice([1.0, 1.0, 0.5, 2.5]))
    # about 4e5 arrivals at most, so the oracle stays quick
    T = float(min(30.0, 4e5 / (n * rate)) * rng.uniform(0.3, 1.0))
    params = workloads.lattice(dim, L, beta, rule, J=J, h=h, init=init, seed=100 + i,
                               T=T, rate=rate)
    tile = [int(rng.integers(1, max(2, x + 2))) for x in L] + [1] * (3 - dim)
    ghost = [int(rng.integers(0, 6)) for _ in range(dim)] + [0] * (3 - dim)
    tuning = dict(tile=tuple(tile), ghost=tuple(ghost),
                  max_sweeps=int(rng.choice([1, 2, 5, 16, 64, 1000])),
                  block=int(rng.choice([64, 128, 256, 512, 768, 1024])))
    return params, tuning


@pytest.mark.parametrize("i", range(N_DRAWS))
def test_random_draw_matches_oracle(torch, i):
    params, tuning = draw(i)
    print(f"draw {i}: {params} {tuning}", file=sys.stderr, flush=True)
    s, t, n, ev, fl = oracle.simulate(params, params["T"])
    try:
        gs, gt, gn, st = aca.simulate(params, params["T"], tuning=tuning)
    except aca.AcaError as e:
        # only a region too large for a workgroup may be refused
        assert e.code == aca.ACA_EINVAL and ("LDS" in str(e) or "65535" in str(e)), str(e)
        return
    assert np.array_equal(gs, s), "spins"
    assert np.array_equal(gt.view(np.uint64), t.view(np.uint64)), "times"
    assert np.array_equal(gn, n), "counts"
    assert st["events"] == ev and st["flips"] == fl


N_AUTO = 24


def draw_auto(i):
    """A lattice of each dimension's larger sizes under the automatic schedule
    (which switches to smaller tiles and wider ghosts for small lattices)."""
    params, _ = draw(i)
    rng = np.random.default_rng(7000 + i)
    dim = params["dim"]
    hi = {1: 30000, 2: 600, 3: 140}[dim]
    L = [int(rng.integers(max(2, hi // 8), hi + 1)) for _ in range(dim)]
    n = int(np.prod(L))
    T = float(min(20.0, 2e6 / (n * params["rate"])) * rng.uniform(0.3, 1.0))
    return dict(params, L=L, T=T)


@pytest.mark.parametrize("i", range(N_AUTO))
def test_random_draw_automatic_schedule(torch, i):
    params = draw_auto(i)
    print(f"auto draw {i}: {params}", file=sys.stderr, flush=True)
    s, t, n, ev, fl = oracle.simulate(params, params["T"])
    gs, gt, gn, st = aca.simulate(params, params["T"])
    assert np.array_equal(gs, s), "spins"
    assert np.array_equal(gt.view(np.uint64), t.view(np.uint64)), "times"
    assert np.array_equal(gn, n), "counts"
    assert st["events"] == ev and st["flips"] == fl
