"""Pins of the oracle's q-th degree neighbourhoods (Section 3, after Fig. 3.5).

neighbors^q(c) applies the nearest-neighbour map q times: the cells within
lattice distance q.  The flip rule reads the spin sum over that set without c.
What fixes the oracle here, independently of its own code:

* the set sizes: the paper prints |neighbors^q(c)| - 1 = 2q(q+1) for the square
  array; 2q on a ring; the octahedral numbers minus one in 3D;
* the stationary law of small rings by enumeration (reversibility for
  H = -J sum over pairs within distance q of s s' - h sum s);
* a pure-Python simulator that finds the neighbours by measuring periodic
  distances (no offset table) and scans for the global minimum;
* q = 1 through the same code equals the nearest-neighbour oracle;
* beta = 0 Metropolis: every arrival flips.
"""
import ctypes
import itertools
import math

import numpy as np
import pytest

import oracle


def P(dim, L, beta, rule="glauber", J=1.0, h=0.0, init="random", seed=1, rate=1.0, q=2):
    return dict(dim=dim, L=list(L), J=J, h=h, beta=beta, rate=rate, rule=rule,
                init=init, seed=seed, range=q)


@pytest.mark.parametrize("q", [1, 2, 3, 4, 5])
def test_set_sizes(q):
    # 2 (z + 1) threshold entries for z = |neighbors^q(c)| - 1
    assert len(oracle.thresholds(2, 1.0, 0.0, 0.3, "glauber", q)) == 2 * (2 * q * (q + 1) + 1)
    assert len(oracle.thresholds(1, 1.0, 0.0, 0.3, "glauber", q)) == 2 * (2 * q + 1)
    if q <= 3:
        octa = (2 * q + 1) * (2 * q * q + 2 * q + 3) // 3          # 7, 25, 63
        assert len(oracle.thresholds(3, 1.0, 0.0, 0.3, "glauber", q)) == 2 * octa


def test_thresholds_follow_the_rule():
    J, h, beta = 0.7, 0.3, 0.4
    thr = oracle.thresholds(2, J, h, beta, "glauber", 2)
    z = 12
    for spin in (-1, 1):
        for total in range(-z, z + 1, 2):
            dE = 2.0 * spin * (J * total + h)
            p = 1.0 / (1.0 + math.exp(beta * dE))
            idx = (total + z) // 2 + (z + 1) * (spin + 1) // 2
            assert thr[idx] == math.floor(p * 2.0 ** 32)


def _periodic_ball(dim, L, q):
    """Neighbours of every cell, found by measuring periodic distances."""
    Ls = list(L) + [1] * (3 - dim)
    N = int(np.prod(Ls))
    coords = [(c % Ls[0], (c // Ls[0]) % Ls[1], c // (Ls[0] * Ls[1])) for c in range(N)]

    def dist(a, b):
        return sum(min(abs(a[d] - b[d]), Ls[d] - abs(a[d] - b[d])) for d in range(3))

    return N, [[j for j in range(N) if j != i and dist(coords[i], coords[j]) <= q]
               for i in range(N)]


def brute_force(params, T):
    dim, q = params["dim"], params["range"]
    N, nb = _periodic_ball(dim, params["L"], q)
    z = len(nb[0])
    thr = oracle.thresholds(dim, params["J"], params["h"], params["beta"], params["rule"], q)
    s, t, n = oracle.init(params)
    s = [int(v) for v in s]
    t = [float(v) for v in t]
    n = [int(v) for v in n]
    while True:
        c = min(range(N), key=lambda i: (t[i], i))
        if not t[c] < T:
            break
        y = oracle.philox(np.array([[n[c], c, 0, 0]]), params["seed"])[0]
        total = sum(s[k] for k in nb[c])
        idx = (total + z) // 2 + (z + 1) * (s[c] + 1) // 2
        if int(y[2]) < int(thr[idx]):
            s[c] = -s[c]
        w = np.array([(int(y[1]) << 32) | int(y[0])], dtype=np.uint64)
        t[c] = t[c] + float(oracle.neg_log_words(w)[0]) / params["rate"]
        n[c] += 1
    return np.array(s, dtype=np.int8), np.array(t), np.array(n, dtype=np.uint32)


@pytest.mark.parametrize("params,T", [
    (P(2, (5, 6), 0.25, "glauber", h=0.2, seed=11), 12.0),
    (P(2, (7, 8), 0.3, "metropolis", J=-0.6, h=0.1, seed=12, q=3), 6.0),
    (P(1, (9,), 0.4, "glauber", seed=13, q=3), 30.0),
    (P(3, (5, 6, 5), 0.12, "metropolis", h=-0.2, seed=14), 3.0),
    (P(2, (6, 5), 0.5, "glauber", init="plus", seed=15, rate=1.7), 9.0),
])
def test_brute_force_identical(params, T):
    s, t, n, ev, fl = oracle.simulate(params, T)
    bs, bt, bn = brute_force(params, T)
    assert np.array_equal(s, bs) and np.array_equal(t, bt) and np.array_equal(n, bn)
    assert ev == int(n.sum())


def test_range_one_is_the_nearest_neighbour_model():
    lib = oracle.lib()
    for params, T in ((P(2, (9, 7), 0.4, seed=21, q=1), 20.0),
                      (P(3, (4, 5, 3), 0.2, "metropolis", h=0.1, seed=22, q=1), 8.0)):
        s, t, n = oracle.init(params)
        s2, t2, n2 = s.copy(), t.copy(), n.copy()
        oracle.run(params, T, s, t, n)
        flips = ctypes.c_uint64(0)
        dims = np.asarray(list(params["L"]) + [1] * (3 - params["dim"]), dtype=np.int32)
        ev = lib.oracle_run_range(params["dim"], oracle._p(dims), 1, params["J"], params["h"],
                                  params["beta"], params["rate"], oracle.RULES[params["rule"]],
                                  params["seed"], T, oracle._p(s2), oracle._p(t2),
                                  oracle._p(n2), ctypes.byref(flips))
        assert ev == int(n.sum())
        assert np.array_equal(s, s2) and np.array_equal(t, t2) and np.array_equal(n, n2)


def test_sides_must_exceed_twice_the_range():
    with pytest.raises(ValueError):
        oracle.simulate(P(2, (4, 9), 0.3, q=2), 1.0)
    with pytest.raises(ValueError):
        oracle.simulate(P(1, (6,), 0.3, q=3), 1.0)


def test_beta_zero_metropolis_flips_every_arrival():
    params = P(2, (11, 8), 0.0, "metropolis", seed=31, q=3)
    s0, _, _ = oracle.init(params)
    s, t, n, ev, fl = oracle.simulate(params, 7.0)
    assert fl == ev
    assert np.array_equal(s, (s0 * np.where(n % 2 == 1, -1, 1)).astype(np.int8))


@pytest.mark.parametrize("L,q,beta,rule,J,h", [
    (5, 2, 0.35, "glauber", 1.0, 0.3),
    (6, 2, 0.3, "metropolis", 0.8, -0.2),
    (7, 3, 0.15, "glauber", 1.0, 0.25),
])
def test_ring_stationary_law_by_enumeration(L, q, beta, rule, J, h):
    """Time-weighted occupancy of a long run vs pi ~ exp(-beta H) with
    H = -J sum_{pairs within distance q} s s' - h sum s."""
    N, nb = _periodic_ball(1, (L,), q)
    states = list(itertools.product((-1, 1), repeat=N))
    index = {s: i for i, s in enumerate(states)}

    def energy(sp):
        e = -h * sum(sp)
        for i in range(N):
            for j in nb[i]:
                if j > i:
                    e -= J * sp[i] * sp[j]
        return e

    E = np.array([energy(s) for s in states])
    pi = np.exp(-beta * (E - E.min()))
    pi /= pi.sum()
    params = P(1, (L,), beta, rule, J, h, seed=4243, q=q)
    s, t, n = oracle.init(params)
    oracle.run(params, 20.0, s, t, n)
    occ = []
    T = 20.0
    while T < 30000.0:
        T += 0.5
        oracle.run(params, T, s, t, n)
        occ.append(index[tuple(int(v) for v in s)])
    occ = np.array(occ)
    hist = np.bincount(occ, minlength=len(states)) / occ.size
    tvd = 0.5 * np.abs(hist - pi).sum()
    assert tvd < 0.05 if N <= 6 else tvd < 0.08
    # power: the nearest-neighbour energy gives a clearly different law
    E1 = np.array([-h * sum(sp) - J * sum(sp[i] * sp[(i + 1) % N] for i in range(N))
                   for sp in states])
    pi1 = np.exp(-beta * (E1 - E1.min()))
    pi1 /= pi1.sum()
    assert 0.5 * np.abs(hist - pi1).sum() > 2 * tvd
