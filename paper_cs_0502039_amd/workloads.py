"""Seeded synthetic workloads for the Poisson-asynchronous Ising array.

This module holds no arithmetic of the method.  It only lists lattice parameter
sets -- geometry, coupling J, field h, inverse temperature beta, update rule,
initial condition, seed and horizon T -- drawn with fixed numpy seeds.  The GPU
library's tests and benchmark and the oracle's golden-value script both take
their inputs from here, so both sides simulate the same lattices.

The paper measures on no public dataset: its runs are Ising lattices with
random initial spins and rate-1 Poisson arrivals (Section 4, appendix), which is
what these generators produce at the sizes the benchmark asks for.

A lattice is a plain dict::

    {"dim": 2, "L": [64, 64], "J": 1.0, "h": 0.0, "beta": 0.4, "rate": 1.0,
     "rule": "glauber", "init": "random", "seed": 1, "T": 100.0}
"""
from __future__ import annotations

import math

import numpy as np

BETA_C_2D = 0.4406868        # critical coupling of the square lattice
BETA_C_3D = 0.2216544        # critical coupling of the simple cubic lattice


def lattice(dim, L, beta, rule="glauber", J=1.0, h=0.0, init="random", seed=1,
            T=1.0, rate=1.0) -> dict:
    return {"dim": int(dim), "L": [int(x) for x in L], "J": float(J), "h": float(h),
            "beta": float(beta), "rate": float(rate), "rule": rule, "init": init,
            "seed": int(seed), "T": float(T)}


def square_64() -> dict:
    """64x64 torus, beta = 0.4, Glauber, random spins, horizon 100 (~4.1e5 arrivals)."""
    return lattice(2, (64, 64), 0.4, "glauber", seed=1, T=100.0)


def square_4096() -> dict:
    """4096x4096 torus at the critical coupling, Glauber, random spins, horizon 200
    (~3.4e9 arrivals)."""
    return lattice(2, (4096, 4096), BETA_C_2D, "glauber", seed=2, T=200.0)


def cubic_256() -> dict:
    """256^3 periodic cube at the 3D critical coupling, h = 0.1, Metropolis, all spins
    +1, horizon 100 (~1.7e9 arrivals)."""
    return lattice(3, (256, 256, 256), BETA_C_3D, "metropolis", h=0.1, init="plus",
                   seed=3, T=100.0)


def batch_512(count: int = 512) -> list[dict]:
    """512 independent tori: side log-uniform in [32, 1024], beta uniform in
    [0.2, 0.6], horizon uniform in [10, 500], Glauber, h = 0, seeds 0..511."""
    rng = np.random.default_rng(4)
    sides = np.rint(np.exp(rng.uniform(math.log(32), math.log(1024), count))).astype(int)
    betas = rng.uniform(0.2, 0.6, count)
    horizons = rng.uniform(10.0, 500.0, count)
    return [lattice(2, (int(s), int(s)), float(b), "glauber", seed=i, T=float(T))
            for i, (s, b, T) in enumerate(zip(sides, betas, horizons))]


def served_stream(count: int = 400, rate_jobs_per_s: float = 1.0) -> list[dict]:
    """A Poisson stream of jobs: 80% 2D tori with side log-uniform in [32, 2048],
    20% 3D cubes with side uniform in {16..128}; beta uniform in [0.15, 0.6];
    Glauber or Metropolis with equal odds; horizon uniform in [10, 1000]; seed
    10^6 + job id.  Each job carries its arrival time "t_arrive" in seconds."""
    rng = np.random.default_rng(5)
    jobs = []
    t = 0.0
    for j in range(count):
        t += float(rng.exponential(1.0 / rate_jobs_per_s))
        if rng.uniform() < 0.8:
            side = int(np.rint(math.exp(rng.uniform(math.log(32), math.log(2048)))))
            dims, L = 2, (side, side)
        else:
            side = int(rng.integers(16, 129))
            dims, L = 3, (side, side, side)
        beta = float(rng.uniform(0.15, 0.6))
        rule = "glauber" if rng.uniform() < 0.5 else "metropolis"
        T = float(rng.uniform(10.0, 1000.0))
        job = lattice(dims, L, beta, rule, seed=10**6 + j, T=T)
        job["t_arrive"] = t
        job["id"] = j
        jobs.append(job)
    return jobs


def square_1024_range(q: int = 2) -> dict:
    """A 1024x1024 torus whose rule reads the q-th degree neighbourhood
    (every cell within lattice distance q: 12 neighbours for q = 2), beta 0.12
    (above the ordering temperature of that coupling range), T = 50."""
    p = lattice(2, (1024, 1024), 0.12 if q == 2 else 0.06, "glauber", seed=8, T=50.0)
    p["range"] = q
    return p


def small_cases() -> list[dict]:
    """Small lattices for element-by-element parity: several tiles, ragged edges,
    every dimension, both rules, odd sides, side 2, fields and couplings of both
    signs."""
    return [
        square_64(),
        lattice(2, (37, 23), 0.44, "metropolis", h=0.1, seed=7, T=30.0),
        lattice(2, (200, 131), BETA_C_2D, "glauber", seed=11, T=20.0),
        lattice(2, (2, 9), 0.5, "glauber", seed=5, T=30.0),
        lattice(2, (2, 2), 0.7, "glauber", h=0.2, seed=1, T=40.0),
        lattice(2, (300, 2), 0.3, "metropolis", J=-1.0, seed=12, T=25.0),
        lattice(2, (129, 257), 0.6, "glauber", init="plus", seed=13, T=15.0),
        lattice(3, (12, 10, 9), BETA_C_3D, "metropolis", h=0.1, init="plus", seed=3, T=20.0),
        lattice(3, (40, 33, 21), 0.3, "glauber", h=-0.05, seed=14, T=12.0),
        lattice(3, (2, 2, 2), 0.25, "metropolis", h=0.15, seed=15, T=30.0),
        lattice(1, (101,), 0.6, "glauber", seed=4, T=40.0),
        lattice(1, (5000,), 1.1, "metropolis", h=0.3, init="minus", seed=16, T=25.0),
        lattice(2, (96, 80), 0.0, "metropolis", seed=17, T=10.0),
        lattice(2, (64, 48), 0.45, "glauber", seed=18, T=5.0, rate=3.0),
    ]
