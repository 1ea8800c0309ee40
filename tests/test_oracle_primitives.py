"""Pins of the oracle's primitives against sources other than itself.

* Philox4x32-10 against rocRAND's independent implementation (run on the host).
* The exponential-gap recipe E(u) = -ln u (Section 3, Eq. (5)) against mpmath at
  120-bit precision, plus its edge cases and the Exp(1) law.
* The flip thresholds (Ising rule of Section 1, probability table of the appendix
  program) against the closed forms evaluated in mpmath.
"""
import math
import os
import shutil
import subprocess

import mpmath as mp
import numpy as np
import pytest
from scipy import stats

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


# ------------------------------------------------------------------ Philox

@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND comparator")
    out = tmp_path_factory.mktemp("rr") / "philox_ref"
    subprocess.run([hipcc, "-O1", "-o", str(out),
                    os.path.join(HERE, "rocrand_philox_ref.cpp")], check=True)
    return str(out)


def test_philox_matches_rocrand(rocrand_ref):
    rng = np.random.default_rng(123)
    rows = []
    # special counters: the two streams the method uses, plus extreme words
    for seed in (0, 1, 2, 3, 2**32 - 1, 2**64 - 1, 0x0123456789ABCDEF):
        rows.append((seed, 0, 0, 0, 0))
        rows.append((seed, 0, 5, 1, 0))
        rows.append((seed, 2**32 - 1, 2**32 - 1, 2**32 - 1, 2**32 - 1))
        rows.append((seed, 17, 4095, 0, 0))
    for _ in range(2000):
        seed = int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2))
        c = rng.integers(0, 2**32, size=4, dtype=np.uint64)
        rows.append((seed, *map(int, c)))
    text = "\n".join(" ".join(str(v) for v in r) for r in rows) + "\n"
    res = subprocess.run([rocrand_ref], input=text, capture_output=True, text=True,
                         check=True)
    want = np.array([[int(v) for v in line.split()] for line in res.stdout.splitlines()],
                    dtype=np.uint64)
    got = np.concatenate([oracle.philox(np.array([r[1:]], dtype=np.uint64), r[0])
                          for r in rows]).astype(np.uint64)
    assert want.shape == got.shape
    assert np.array_equal(want, got)


def test_philox_is_a_function_of_counter_and_key():
    ctr = np.array([[3, 9, 0, 0], [3, 9, 1, 0], [4, 9, 0, 0], [3, 10, 0, 0]])
    a = oracle.philox(ctr, 77)
    b = oracle.philox(ctr, 77)
    c = oracle.philox(ctr, 78)
    assert np.array_equal(a, b)
    assert len({tuple(r) for r in a}) == 4          # distinct counters differ
    assert not np.array_equal(a, c)                 # the key matters


# ------------------------------------------------------------------ u and -ln u

mp.mp.prec = 120


def _ulp_err(got: float, u: float) -> float:
    exact = -mp.log(mp.mpf(u))
    return float(abs(mp.mpf(got) - exact) / math.ulp(float(exact)))


def test_uniform_mapping_exact_and_open():
    w = np.array([0, 1, (1 << 12) - 1, 1 << 12, (1 << 64) - 1, 1 << 63], dtype=np.uint64)
    u = oracle.uniform_words(w)
    assert u[0] == 2.0 ** -53 and u[1] == 2.0 ** -53 and u[2] == 2.0 ** -53
    assert u[3] == 3 * 2.0 ** -53
    assert u[4] == 1.0 - 2.0 ** -53
    assert u[5] == 0.5 + 2.0 ** -53
    assert np.all((u > 0) & (u < 1))


def test_ln2_split_against_mpmath():
    hi, lo = oracle.ln2_split()
    ln2 = mp.log(2)
    m, e = math.frexp(hi)
    assert (int(m * 2 ** 53) & ((1 << 14) - 1)) == 0          # head has <= 39 bits
    assert lo == float(ln2 - mp.mpf(hi))                       # tail correctly rounded
    assert abs(mp.mpf(hi) + mp.mpf(lo) - ln2) < mp.mpf(2) ** -95


def test_neg_log_accuracy_random():
    rng = np.random.default_rng(7)
    w = rng.integers(0, 2**64, size=20000, dtype=np.uint64)
    e = oracle.neg_log_words(w)
    u = oracle.uniform_words(w)
    worst = max(_ulp_err(float(a), float(b)) for a, b in zip(e, u))
    assert worst <= 2.0, worst


def test_neg_log_accuracy_edges():
    # extremes of u, exact powers of two, both sides of the sqrt(2) split,
    # and u next to 1/2, where the head and the series nearly cancel
    ws = [0, (1 << 64) - 1, 1 << 63, (1 << 63) - (1 << 12), 1 << 62, 1 << 13]
    s2 = math.sqrt(2.0) / 2
    for u in (s2 * (1 - 1e-12), s2 * (1 + 1e-12), 0.5 * (1 + 1e-9), 0.5 * (1 - 1e-9),
              0.25 * math.sqrt(2.0), 1 - 1e-6, 1e-10):
        m = int(u * 2.0 ** 52)
        ws.append(m << 12)
    w = np.array(ws, dtype=np.uint64)
    e = oracle.neg_log_words(w)
    u = oracle.uniform_words(w)
    for a, b in zip(e, u):
        assert a > 0.0
        assert _ulp_err(float(a), float(b)) <= 2.0
    assert e[0] == pytest.approx(53 * math.log(2), rel=1e-15)   # u = 2^-53
    assert e[1] == pytest.approx(2.0 ** -53, rel=1e-12)          # u = 1 - 2^-53


def test_neg_log_is_exponential_one():
    rng = np.random.default_rng(11)
    w = rng.integers(0, 2**64, size=200000, dtype=np.uint64)
    e = oracle.neg_log_words(w)
    ks = stats.kstest(e, "expon")
    assert ks.pvalue > 1e-3
    assert abs(e.mean() - 1.0) < 5 * 1.0 / math.sqrt(e.size)


# ------------------------------------------------------------------ thresholds

def _p_exact(rule, beta, J, h, spin, total):
    dE = 2 * spin * (mp.mpf(J) * total + mp.mpf(h))
    if rule == "glauber":
        return 1 / (1 + mp.exp(mp.mpf(beta) * dE))
    return mp.mpf(1) if dE <= 0 else mp.exp(-mp.mpf(beta) * dE)


@pytest.mark.parametrize("dim", [1, 2, 3])
@pytest.mark.parametrize("rule", ["glauber", "metropolis"])
@pytest.mark.parametrize("beta,J,h", [(0.4, 1.0, 0.0), (0.4406868, 1.0, 0.0),
                                      (0.2216544, 1.0, 0.1), (1.3, -0.7, 0.25),
                                      (0.05, 2.0, -1.5)])
def test_thresholds_against_closed_form(dim, rule, beta, J, h):
    z = 2 * dim
    thr = oracle.thresholds(dim, J, h, beta, rule)
    assert thr.size == 2 * (z + 1)
    for spin in (-1, 1):
        for total in range(-z, z + 1, 2):
            idx = (total + z) // 2 + (z + 1) * (spin + 1) // 2
            p = _p_exact(rule, beta, J, h, spin, total)
            if p >= 1:
                assert thr[idx] == 2 ** 32
                continue
            scaled = p * 2 ** 32
            fl = int(mp.floor(scaled))
            if abs(scaled - fl) > 1e-6 and abs(scaled - fl - 1) > 1e-6:
                assert int(thr[idx]) == fl, (spin, total)
            else:
                assert abs(int(thr[idx]) - fl) <= 1


def test_thresholds_special_values():
    # beta = 0: Glauber flips with probability exactly 1/2, Metropolis always
    assert np.all(oracle.thresholds(2, 1.0, 0.3, 0.0, "glauber") == 2 ** 31)
    assert np.all(oracle.thresholds(3, 1.0, 0.3, 0.0, "metropolis") == 2 ** 32)
    # Metropolis always accepts moves that do not raise the energy
    thr = oracle.thresholds(2, 1.0, 0.0, 0.7, "metropolis")
    z = 4
    for spin in (-1, 1):
        for total in range(-z, z + 1, 2):
            idx = (total + z) // 2 + (z + 1) * (spin + 1) // 2
            if spin * total <= 0:
                assert thr[idx] == 2 ** 32
    # Glauber symmetric under (s, sum) -> (-s, -sum) at h = 0, and p + p' = 1
    thr = oracle.thresholds(2, 1.0, 0.0, 0.4406868, "glauber")
    for i in range(5):
        assert thr[i] == thr[9 - i]
        assert abs(int(thr[i]) + int(thr[4 - i]) - 2 ** 32) <= 1
