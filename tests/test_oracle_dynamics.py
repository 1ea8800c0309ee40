"""Pins of the oracle's dynamics against exact mathematics.

The oracle applies arrivals in increasing (time, index) order (the unique
trajectory of Section 3).  These tests check it against results that do not
come from the oracle:

* exact stationary laws of 2x2 and 3x3 periodic lattices, by enumerating all
  states (time averages of the oracle's trajectory must match pi ~ exp(-beta H));
* exact transient laws expm(Q t) P0 of the continuous-time chain whose generator
  Q is built here from the Ising rule (Section 1: transient behaviour matters);
* closed forms: beta = 0 (Metropolis flips at every arrival, Glauber with
  probability 1/2), Poisson arrival counts, the per-cell arrival clock;
* Onsager's energy and Yang's magnetisation of the 2D lattice at long times;
* a pure-Python brute-force simulator on tiny lattices (global minimum by scan);
* the paper's parallel schedules (Fig. 3.2 rounds, Fig. 3.4 tiles) reaching the
  identical state, and the Section 4 efficiency constants 0.121 (2D) and 0.247 (1D).

Each statistical test also checks that a plausible mistake (flipped field sign,
exchanged rule) would move the observable far outside the tolerance.
"""
import itertools
import math

import numpy as np
import pytest
from scipy import linalg, special, stats

import oracle


def P(dim, L, beta, rule="glauber", J=1.0, h=0.0, init="random", seed=1, rate=1.0):
    return dict(dim=dim, L=list(L), J=J, h=h, beta=beta, rate=rate, rule=rule,
                init=init, seed=seed)


# ------------------------------------------------------------ exact small chains

def _slots(dim, L):
    """Neighbour slots of every cell (index x + Lx (y + Ly z)), with multiplicity."""
    Ls = list(L) + [1] * (3 - dim)
    N = int(np.prod(Ls))
    nb = []
    for c in range(N):
        x, y, z = c % Ls[0], (c // Ls[0]) % Ls[1], c // (Ls[0] * Ls[1])
        co = [x, y, z]
        row = []
        for d in range(dim):
            for step in (1, -1):
                q = list(co)
                q[d] = (q[d] + step) % Ls[d]
                row.append(q[0] + Ls[0] * (q[1] + Ls[1] * q[2]))
        nb.append(row)
    return N, nb


def _energy(spins, nb, dim, J, h):
    # bonds along +e_d only (slot 2d), so each bond once (twice at side 2,
    # matching the slot multiplicity of the dynamics)
    e = 0.0
    for c, row in enumerate(nb):
        for d in range(dim):
            e -= J * spins[c] * spins[row[2 * d]]
    return e - h * sum(spins)


def _flip_prob(rule, beta, dE):
    if rule == "glauber":
        return 1.0 / (1.0 + math.exp(beta * dE))
    return 1.0 if dE <= 0 else math.exp(-beta * dE)


def exact_chain(dim, L, beta, rule, J, h):
    """States (as +/-1 tuples), stationary law and generator Q (columns = from)."""
    N, nb = _slots(dim, L)
    states = list(itertools.product((-1, 1), repeat=N))
    index = {s: i for i, s in enumerate(states)}
    E = np.array([_energy(s, nb, dim, J, h) for s in states])
    pi = np.exp(-beta * (E - E.min()))
    pi /= pi.sum()
    M = len(states)
    Q = np.zeros((M, M))
    for i, s in enumerate(states):
        for c in range(N):
            total = sum(s[k] for k in nb[c])
            dE = 2 * s[c] * (J * total + h)
            r = _flip_prob(rule, beta, dE)
            t = list(s)
            t[c] = -t[c]
            j = index[tuple(t)]
            Q[j, i] += r
            Q[i, i] -= r
    return states, index, pi, Q, E


def _state_key(s):
    return tuple(int(v) for v in s)


def time_average(params, T_end, dt, burn, fn):
    s, t, n = oracle.init(params)
    oracle.run(params, burn, s, t, n)
    vals = []
    T = burn
    while T < T_end:
        T += dt
        oracle.run(params, T, s, t, n)
        vals.append(fn(s))
    return np.array(vals)


def _batch_sigma(x, nb=50):
    b = np.array_split(x, nb)
    means = np.array([v.mean() for v in b])
    return means.std(ddof=1) / math.sqrt(nb)


CASES = [
    (2, (2, 2), 0.45, "glauber", 1.0, 0.3),
    (2, (2, 2), 0.45, "metropolis", 1.0, 0.3),
    (2, (3, 3), 0.3, "glauber", 1.0, -0.2),
    (2, (3, 3), 0.3, "metropolis", 0.8, 0.25),
    (1, (5,), 0.7, "glauber", 1.0, 0.2),
    (3, (2, 2, 2), 0.25, "metropolis", 1.0, 0.15),
]


@pytest.mark.parametrize("dim,L,beta,rule,J,h", CASES)
def test_stationary_law_by_enumeration(dim, L, beta, rule, J, h):
    states, index, pi, Q, E = exact_chain(dim, L, beta, rule, J, h)
    N = len(states[0])
    params = P(dim, L, beta, rule, J, h, seed=4242)
    occ = time_average(params, 40000.0, 0.5, 20.0,
                       lambda s: index[_state_key(s)])
    # exact expectations of energy and magnetisation vs time averages
    Es = E[occ]
    Ms = np.array([sum(states[i]) for i in occ], dtype=float)
    Mexact = sum(p * sum(st) for p, st in zip(pi, states))
    Eexact = float(np.dot(pi, E))
    for obs, exact in ((Es, Eexact), (Ms, Mexact)):
        sig = _batch_sigma(obs)
        assert abs(obs.mean() - exact) < 5 * sig + 1e-3, (obs.mean(), exact, sig)
    # the full law: total variation distance from pi
    hist = np.bincount(occ, minlength=len(states)) / occ.size
    tvd = 0.5 * np.abs(hist - pi).sum()
    assert tvd < 0.04 if N <= 5 else tvd < 0.12
    # power: the same chain with the field reversed has a law that is far away
    if h != 0:
        _, _, pi_bad, _, E_bad = exact_chain(dim, L, beta, rule, J, -h)
        Mbad = sum(p * sum(st) for p, st in zip(pi_bad, states))
        assert abs(Mbad - Mexact) > 10 * _batch_sigma(Ms)


@pytest.mark.parametrize("dim,L,beta,rule,J,h,tq", [
    (2, (2, 2), 0.6, "glauber", 1.0, 0.4, 0.35),
    (2, (2, 2), 0.6, "metropolis", 1.0, 0.4, 0.35),
    (2, (2, 2), 0.6, "glauber", 1.0, 0.4, 1.5),
    (1, (3,), 0.9, "metropolis", 1.0, -0.5, 0.8),
])
def test_transient_law_expm(dim, L, beta, rule, J, h, tq):
    """Ensemble over seeds at time tq vs expm(Q tq) P0 with P0 uniform (iid fair spins)."""
    states, index, pi, Q, E = exact_chain(dim, L, beta, rule, J, h)
    M = len(states)
    p0 = np.full(M, 1.0 / M)
    pt = linalg.expm(Q * tq) @ p0
    nseeds = 30000
    counts = np.zeros(M)
    for seed in range(nseeds):
        params = P(dim, L, beta, rule, J, h, seed=seed + 1000)
        s, t, n, ev, fl = oracle.simulate(params, tq)
        counts[index[_state_key(s)]] += 1
    chi2 = ((counts - nseeds * pt) ** 2 / (nseeds * pt)).sum()
    pval = stats.chi2.sf(chi2, M - 1)
    assert pval > 1e-4, (chi2, pval)
    # power: the other rule's transient law is rejected
    other = "metropolis" if rule == "glauber" else "glauber"
    _, _, _, Qo, _ = exact_chain(dim, L, beta, other, J, h)
    po = linalg.expm(Qo * tq) @ p0
    chi2o = ((counts - nseeds * po) ** 2 / (nseeds * po)).sum()
    assert stats.chi2.sf(chi2o, M - 1) < 1e-6


def test_transient_from_all_plus_3x3():
    """3x3 (512 states) started all +1: law of the magnetisation at t = 0.6."""
    states, index, pi, Q, E = exact_chain(2, (3, 3), 0.5, "glauber", 1.0, -0.3)
    M = len(states)
    p0 = np.zeros(M)
    p0[index[(1,) * 9]] = 1.0
    pt = linalg.expm(Q * 0.6) @ p0
    mags = np.array([sum(st) for st in states])
    want = np.array([pt[mags == m].sum() for m in range(-9, 10, 2)])
    counts = np.zeros(10)
    nseeds = 20000
    for seed in range(nseeds):
        params = P(2, (3, 3), 0.5, "glauber", 1.0, -0.3, init="plus", seed=seed)
        s, *_ = oracle.simulate(params, 0.6)
        counts[(int(s.sum()) + 9) // 2] += 1
    keep = want * nseeds > 5
    chi2 = ((counts[keep] - nseeds * want[keep]) ** 2 / (nseeds * want[keep])).sum()
    assert stats.chi2.sf(chi2, keep.sum() - 1) > 1e-4


# ------------------------------------------------------------ closed forms

def test_beta_zero_metropolis_flips_every_arrival():
    params = P(2, (32, 48), 0.0, "metropolis", seed=5)
    s0, _, _ = oracle.init(params)
    s, t, n, ev, fl = oracle.simulate(params, 7.5)
    sign = np.where(n % 2 == 0, 1, -1).astype(np.int8)
    assert np.array_equal(s, s0 * sign)
    assert ev == fl == int(n.sum())


def test_beta_zero_glauber_half_flips():
    params = P(2, (128, 128), 0.0, "glauber", seed=6)
    s0, _, _ = oracle.init(params)
    T = 0.8
    s, t, n, ev, fl = oracle.simulate(params, T)
    assert np.array_equal(s[n == 0], s0[n == 0])
    frac = float((s == s0).mean())
    want = math.exp(-T) + (1 - math.exp(-T)) / 2
    assert abs(frac - want) < 5 * math.sqrt(want * (1 - want) / s.size)
    assert abs(fl / ev - 0.5) < 5 * 0.5 / math.sqrt(ev)


def test_initial_state_law():
    params = P(2, (200, 200), 0.3, seed=9)
    s, t, n = oracle.init(params)
    assert set(np.unique(s)) == {-1, 1} and np.all(n == 0)
    assert abs(s.mean()) < 5 / math.sqrt(s.size)
    assert stats.kstest(t, "expon").pvalue > 1e-3     # first arrival ~ Exp(rate)
    sp, _, _ = oracle.init(dict(params, init="plus"))
    sm, _, _ = oracle.init(dict(params, init="minus"))
    assert np.all(sp == 1) and np.all(sm == -1)
    t2 = oracle.init(dict(params, rate=4.0))[1]
    assert np.array_equal(t2, t / 4.0)                 # exact: division by 4


@pytest.mark.parametrize("rule,beta,h", [("glauber", 0.7, 0.3), ("metropolis", 0.5, -0.4),
                                          ("glauber", 1.3, -0.25)])
@pytest.mark.parametrize("init", ["plus", "minus"])
def test_independent_spins_closed_form(rule, beta, h, init):
    """J = 0: every cell is a two-state chain of its own.  An arrival reverses a
    +1 spin with probability a = thr[+]/2^32 and a -1 spin with b = thr[-]/2^32
    (Section 2's rule with the field alone), so at unit rate
    P(s = +1, t) = pi + (P0 - pi) exp(-(a + b) t), pi = b / (a + b).
    A sign slip in the field or the spin side of the table fails this."""
    N, T = 40000, 1.2
    params = P(1, (N,), beta, rule, J=0.0, h=h, init=init, seed=77)
    thr = oracle.thresholds(1, 0.0, h, beta, rule).astype(np.float64) / 2.0 ** 32
    z = 2
    a, b = thr[z + 1], thr[0]           # spin +1 entries follow the spin -1 ones
    assert np.all(thr[z + 1:] == a) and np.all(thr[:z + 1] == b)
    pi = b / (a + b)
    p0 = 1.0 if init == "plus" else 0.0
    want = pi + (p0 - pi) * math.exp(-(a + b) * T)
    s, _, _, _, _ = oracle.simulate(params, T)
    got = float(np.mean(s == 1))
    sigma = math.sqrt(want * (1.0 - want) / N)
    assert abs(got - want) < 5.0 * sigma, (got, want, sigma)
    # power: the field's sign swapped gives a clearly different value
    swapped = (1.0 - pi) + (p0 - (1.0 - pi)) * math.exp(-(a + b) * T)
    assert abs(swapped - want) > 20.0 * sigma


def test_poisson_counts_and_cell_clock():
    params = P(2, (64, 64), 0.4406868, seed=2)
    T = 30.0
    s, t, n, ev, fl = oracle.simulate(params, T)
    assert ev == int(n.sum())
    assert np.all(t >= T)
    # counts ~ Poisson(T): chi-square on binned pmf
    ks = np.arange(0, 80)
    pmf = stats.poisson.pmf(ks, T)
    obs = np.bincount(n, minlength=80)[:80].astype(float)
    keep = pmf * n.size > 5
    chi2 = ((obs[keep] - n.size * pmf[keep]) ** 2 / (n.size * pmf[keep])).sum()
    assert stats.chi2.sf(chi2, keep.sum() - 1) > 1e-4
    # time and count of every cell follow from its own draws alone
    tc, nc = oracle.cell_clock(params, np.arange(n.size), T)
    assert np.array_equal(tc, t) and np.array_equal(nc, n)


def test_rate_scales_time():
    """With rate 2 the process is the rate-1 process with times halved."""
    a = P(2, (16, 16), 0.5, seed=3)
    b = dict(a, rate=2.0)
    s1, t1, n1, *_ = oracle.simulate(a, 10.0)
    s2, t2, n2, *_ = oracle.simulate(b, 5.0)
    assert np.array_equal(n1, n2)
    assert np.array_equal(s1, s2)
    assert np.allclose(t1 / 2.0, t2, rtol=1e-13)


def test_chunked_advance_is_identical():
    params = P(2, (40, 24), 0.44, "metropolis", h=0.05, seed=12)
    s, t, n, *_ = oracle.simulate(params, 25.0)
    s2, t2, n2 = oracle.init(params)
    for T in (0.0, 3.3, 3.3, 10.0, 17.25, 25.0):
        oracle.run(params, T, s2, t2, n2)
    assert np.array_equal(s, s2) and np.array_equal(t, t2) and np.array_equal(n, n2)


def test_zero_temperature_metropolis_never_raises_energy():
    params = P(2, (32, 32), 50.0, "metropolis", h=0.05, seed=21)
    _, nb = _slots(2, (32, 32))
    nbx = np.array([row[0] for row in nb])
    nby = np.array([row[2] for row in nb])

    def energy(s):
        s = s.astype(np.int64)
        return float(-(s * s[nbx]).sum() - (s * s[nby]).sum() - 0.05 * s.sum())

    s, t, n = oracle.init(params)
    last = energy(s)
    for T in np.arange(0.25, 20.0, 0.25):
        oracle.run(params, T, s, t, n)
        e = energy(s)
        assert e <= last + 1e-9
        last = e


# ------------------------------------------------------------ 2D thermodynamics

def onsager_energy(beta, J=1.0):
    k = 2 * math.sinh(2 * beta * J) / math.cosh(2 * beta * J) ** 2
    K = special.ellipk(k * k)
    th = math.tanh(2 * beta * J)
    return -J / math.tanh(2 * beta * J) * (1 + 2 / math.pi * (2 * th * th - 1) * K)


def test_onsager_closed_form_values():
    assert onsager_energy(0.4) == pytest.approx(-1.10608, abs=2e-5)
    assert onsager_energy(0.6) == pytest.approx(-1.90909, abs=2e-5)
    # at the critical point the energy tends to -sqrt(2) (k -> 1, K(k) diverges
    # while its prefactor vanishes)
    assert onsager_energy(0.44068) == pytest.approx(-math.sqrt(2), abs=2e-3)


def _bond_energy(L):
    idx = np.arange(L * L).reshape(L, L)
    right = np.roll(idx, -1, axis=1).ravel()
    down = np.roll(idx, -1, axis=0).ravel()

    def e(s):
        s = s.astype(np.int64)
        return float(-(s * s[right]).sum() - (s * s[down]).sum()) / s.size
    return e


@pytest.mark.parametrize("rule", ["glauber", "metropolis"])
def test_onsager_energy_long_time(rule):
    L = 64
    params = P(2, (L, L), 0.4, rule, seed=31)
    e = time_average(params, 1500.0, 5.0, 300.0, _bond_energy(L))
    sig = _batch_sigma(e, 20)
    assert abs(e.mean() - onsager_energy(0.4)) < 5 * sig + 0.01, (e.mean(), sig)


def test_yang_magnetisation_from_all_plus():
    L = 64
    beta = 0.6
    params = P(2, (L, L), beta, "glauber", init="plus", seed=32)
    m = time_average(params, 400.0, 4.0, 100.0, lambda s: float(s.mean()))
    yang = (1 - math.sinh(2 * beta) ** -4) ** 0.125
    assert abs(m.mean() - yang) < 0.01, (m.mean(), yang)
    e = time_average(params, 300.0, 4.0, 100.0, _bond_energy(L))
    assert abs(e.mean() - onsager_energy(beta)) < 0.01


# ------------------------------------------------------------ brute force

def brute_force(params, T):
    """Global minimum by linear scan, one arrival at a time (tiny lattices only)."""
    dim = params["dim"]
    N, nb = _slots(dim, params["L"])
    z = 2 * dim
    thr = oracle.thresholds(dim, params["J"], params["h"], params["beta"], params["rule"])
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
    return (np.array(s, dtype=np.int8), np.array(t), np.array(n, dtype=np.uint32))


@pytest.mark.parametrize("params,T", [
    (P(2, (2, 2), 0.7, "glauber", h=0.2, seed=1), 40.0),
    (P(2, (3, 4), 0.3, "metropolis", J=-1.0, h=0.1, seed=2), 15.0),
    (P(1, (2,), 0.5, "glauber", seed=3), 50.0),
    (P(1, (7,), 0.5, "metropolis", h=-0.3, seed=4), 20.0),
    (P(3, (2, 3, 2), 0.2, "glauber", h=0.3, seed=5), 10.0),
    (P(2, (5, 2), 0.9, "metropolis", init="minus", seed=6, rate=2.5), 8.0),
])
def test_brute_force_identical(params, T):
    s, t, n, ev, fl = oracle.simulate(params, T)
    bs, bt, bn = brute_force(params, T)
    assert np.array_equal(s, bs) and np.array_equal(t, bt) and np.array_equal(n, bn)


def test_equal_times_resolved_by_index():
    """Force exact ties: every cell gets the same time; the smaller index goes first."""
    params = P(2, (4, 4), 0.8, "glauber", h=0.1, seed=8)
    s, t, n = oracle.init(params)
    t[:] = 0.5
    s1, t1, n1 = s.copy(), t.copy(), n.copy()
    oracle.run(params, 30.0, s1, t1, n1)
    # brute force from the same tied state
    N, nb = _slots(2, (4, 4))
    thr = oracle.thresholds(2, 1.0, 0.1, 0.8, "glauber")
    S, Tt, Nn = [int(v) for v in s], [0.5] * N, [0] * N
    while True:
        c = min(range(N), key=lambda i: (Tt[i], i))
        if not Tt[c] < 30.0:
            break
        y = oracle.philox(np.array([[Nn[c], c, 0, 0]]), 8)[0]
        total = sum(S[k] for k in nb[c])
        idx = (total + 4) // 2 + 5 * (S[c] + 1) // 2
        if int(y[2]) < int(thr[idx]):
            S[c] = -S[c]
        w = np.array([(int(y[1]) << 32) | int(y[0])], dtype=np.uint64)
        Tt[c] += float(oracle.neg_log_words(w)[0])
        Nn[c] += 1
    assert np.array_equal(s1, np.array(S, dtype=np.int8))
    assert np.array_equal(n1, np.array(Nn, dtype=np.uint32))
    s2, t2, n2 = s.copy(), t.copy(), n.copy()
    oracle.run_rounds(params, 30.0, s2, t2, n2)
    assert np.array_equal(s1, s2) and np.array_equal(t1, t2) and np.array_equal(n1, n2)


# ------------------------------------------------------------ parallel schedules

SCHED_CASES = [
    (P(2, (64, 64), 0.4, "glauber", seed=1), 100.0),
    (P(2, (37, 23), 0.44, "metropolis", h=0.1, seed=7), 30.0),
    (P(3, (12, 10, 9), 0.2216544, "metropolis", h=0.1, init="plus", seed=3), 20.0),
    (P(1, (101,), 0.6, "glauber", seed=4), 40.0),
    (P(2, (2, 9), 0.5, "glauber", seed=5), 30.0),
]


@pytest.mark.parametrize("params,T", SCHED_CASES)
def test_synchronous_rounds_identical(params, T):
    s, t, n, ev, fl = oracle.simulate(params, T)
    s2, t2, n2 = oracle.init(params)
    ev2, rounds, fl2, rec = oracle.run_rounds(params, T, s2, t2, n2)
    assert (ev2, fl2) == (ev, fl)
    assert np.array_equal(s, s2) and np.array_equal(t, t2) and np.array_equal(n, n2)
    assert rec.sum() == ev


@pytest.mark.parametrize("params,T", SCHED_CASES)
@pytest.mark.parametrize("tile,rounds", [((8, 8, 4), 1 << 30), ((16, 5, 3), 3),
                                         ((64, 64, 64), 1 << 30), ((7, 64, 2), 1)])
def test_tiled_frozen_halo_identical(params, T, tile, rounds):
    s, t, n, ev, fl = oracle.simulate(params, T)
    s2, t2, n2 = oracle.init(params)
    ev2, fl2, passes, visits, nr = oracle.run_tiled(params, T, s2, t2, n2, tile, rounds)
    assert (ev2, fl2) == (ev, fl)
    assert np.array_equal(s, s2) and np.array_equal(t, t2) and np.array_equal(n, n2)


def test_round_one_efficiency_is_one_over_z_plus_one():
    """First round: a cell passes iff its first arrival is the smallest of z+1 iid times."""
    for dim, L in ((1, (100000,)), (2, (300, 300)), (3, (48, 48, 48))):
        params = P(dim, L, 0.0, seed=17)
        s, t, n = oracle.init(params)
        _, rounds, _, rec = oracle.run_rounds(params, 30.0, s, t, n, times_only=True,
                                              max_record=2)
        N = s.size
        z = 2 * dim
        frac = rec[0] / N
        assert abs(frac - 1 / (z + 1)) < 6 * math.sqrt(1 / (z + 1) / N), (dim, frac)


@pytest.mark.parametrize("dim,L,T,paper", [(2, (256, 256), 60.0, 0.121),
                                           (1, (65536,), 300.0, 0.247)])
def test_time_only_efficiency_matches_section4(dim, L, T, paper):
    """Section 4: fraction of cells passing the test per round, large arrays."""
    params = P(dim, L, 0.0, seed=19)
    s, t, n = oracle.init(params)
    ev, rounds, _, rec = oracle.run_rounds(params, T, s, t, n, times_only=True,
                                           max_record=1 << 16)
    N = s.size
    steady = rec[rounds // 4: rounds * 3 // 4] / N
    assert abs(steady.mean() - paper) < 0.004, steady.mean()
    assert abs(ev / N - T) < 0.05 * T   # about one arrival per unit time per cell


@pytest.mark.parametrize("params,T", SCHED_CASES)
@pytest.mark.parametrize("tile,ghost,rounds", [((64, 64, 16), (4, 4, 2), 32),
                                               ((16, 8, 8), (3, 2, 1), 5),
                                               ((7, 5, 3), (2, 2, 1), 1 << 30),
                                               ((9, 9, 9), (0, 0, 0), 1)])
def test_ghost_merge_schedule_identical(params, T, tile, ghost, rounds):
    """The GPU library's launch schedule (all tiles against one snapshot, ghost
    zones, copies merged by most arrivals applied) reaches the heap's state."""
    s, t, n, ev, fl = oracle.simulate(params, T)
    s2, t2, n2 = oracle.init(params)
    ev2, launches, nr = oracle.run_ghost_merge(params, T, s2, t2, n2, tile, ghost, rounds)
    assert ev2 == ev
    assert np.array_equal(s, s2) and np.array_equal(t, t2) and np.array_equal(n, n2)


def test_ghost_copies_must_be_merged():
    """Writing back only owned copies loses consistency (a ghost copy can run ahead
    of its owner and an owned neighbour may rely on it): spins then differ."""
    params = P(2, (200, 131), 0.4406868, seed=11)
    s, t, n, ev, fl = oracle.simulate(params, 20.0)
    s2, t2, n2 = oracle.init(params)
    oracle.run_ghost_merge(params, 20.0, s2, t2, n2, (64, 64), (4, 4), 32,
                           merge_ghosts=False)
    assert np.array_equal(t, t2) and np.array_equal(n, n2)   # clocks never depend on spins
    assert not np.array_equal(s, s2)


def test_frames_beta_zero_metropolis_closed_form():
    """Fig. 3.7 frames at beta = 0 under Metropolis: every arrival flips, so the
    spin at time tau is s0 (-1)^n(tau), with n(tau) the closed-form count of the
    cell's arrivals before tau; the frame at the horizon is the final state."""
    p = P(2, (23, 17), 0.0, "metropolis", seed=31)
    s, t, n = oracle.init(p)
    s0 = s.copy()
    cells = np.arange(s.size, dtype=np.uint32)
    fr = oracle.frames(p, 0.0, 6.0, 0.75, 0, 12, s, t, n)
    assert sorted(fr) == list(range(1, 9))          # 0.75 .. 6.0; k = 0 is not after 0
    for k, img in fr.items():
        _, nk = oracle.cell_clock(p, cells, k * 0.75)
        want = (s0 * np.where(nk % 2 == 1, -1, 1)).astype(np.int8)
        assert np.array_equal(img, want), k
    assert np.array_equal(fr[8], s)
    # continuing from the horizon: the next frames, and none before 6.0 again
    fr2 = oracle.frames(p, 6.0, 9.0, 0.75, 0, 20, s, t, n)
    assert sorted(fr2) == list(range(9, 13))
    _, nk = oracle.cell_clock(p, cells, 9.0)
    assert np.array_equal(fr2[12], (s0 * np.where(nk % 2 == 1, -1, 1)).astype(np.int8))
