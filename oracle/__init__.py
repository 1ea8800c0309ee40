"""Serial CPU oracle for the Poisson-asynchronous Ising array (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It never imports the GPU library and the
GPU library never imports it; the two are independent implementations of one
written contract.

``run`` is the oracle proper: every arrival with time < T is applied in
increasing (time, cell index) order, the one trajectory that the conservative
algorithms of Section 3 (Fig. 3.1, 3.2, 3.4) are shown to produce.  The other
entry points expose its primitives (Philox4x32-10, the exponential-gap recipe,
the flip thresholds) for pinning, and serial emulations of the paper's parallel
schedules (``run_rounds``, ``run_tiled``).

Lattice parameters are plain dicts, as produced by the workload generators::

    {"dim": 2, "L": [64, 64], "J": 1.0, "h": 0.0, "beta": 0.4, "rate": 1.0,
     "rule": "glauber" | "metropolis", "init": "random" | "plus" | "minus",
     "seed": 1}

An optional "range": q > 1 selects the q-th degree neighbourhood (Section 3,
after Fig. 3.5): the rule reads the spins of every cell within lattice
distance q (every side must exceed 2q).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SOURCES = ("aca_oracle.c", "aca_sched.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_LOCK = threading.Lock()
_LIB = None

RULES = {"glauber": 0, "metropolis": 1}
INITS = {"random": 0, "plus": 1, "minus": 2}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: -O2, no FP contraction, no fast-math."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES]
    if not force and os.path.exists(_LIB_PATH):
        newest = max(os.path.getmtime(s) for s in srcs)
        if os.path.getmtime(_LIB_PATH) >= newest:
            return _LIB_PATH
    tmp = _LIB_PATH + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-fvisibility=hidden", "-o", tmp, *srcs, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib() -> ctypes.CDLL:
    global _LIB
    with _LOCK:
        if _LIB is None:
            build(force=False)
            L = ctypes.CDLL(_LIB_PATH)
            P = ctypes.c_void_p
            i32, i64, u64, f64 = (ctypes.c_int, ctypes.c_int64, ctypes.c_uint64,
                                  ctypes.c_double)
            L.oracle_philox.argtypes = [P, u64, P, i64]
            L.oracle_philox.restype = None
            L.oracle_neg_log_words.argtypes = [P, P, i64]
            L.oracle_neg_log_words.restype = None
            L.oracle_uniform_words.argtypes = [P, P, i64]
            L.oracle_uniform_words.restype = None
            L.oracle_ln2_split.argtypes = [P, P]
            L.oracle_ln2_split.restype = None
            L.oracle_thresholds.argtypes = [i32, f64, f64, f64, i32, P]
            L.oracle_thresholds.restype = i32
            L.oracle_init.argtypes = [i32, P, f64, i32, u64, P, P, P]
            L.oracle_init.restype = i32
            L.oracle_run.argtypes = [i32, P, f64, f64, f64, f64, i32, u64, f64,
                                     P, P, P, P]
            L.oracle_run.restype = i64
            L.oracle_thresholds_range.argtypes = [i32, i32, f64, f64, f64, i32, P]
            L.oracle_thresholds_range.restype = i32
            L.oracle_run_range.argtypes = [i32, P, i32, f64, f64, f64, f64, i32, u64, f64,
                                           P, P, P, P]
            L.oracle_run_range.restype = i64
            L.oracle_cell_clock.argtypes = [u64, f64, P, i64, f64, P, P]
            L.oracle_cell_clock.restype = None
            L.oracle_run_rounds.argtypes = [i32, P, f64, f64, f64, f64, i32, u64,
                                            f64, i32, P, P, P, P, i64, P, P]
            L.oracle_run_rounds.restype = i64
            L.oracle_run_tiled.argtypes = [i32, P, f64, f64, f64, f64, i32, u64,
                                           f64, P, i64, i64, P, P, P, P, P]
            L.oracle_run_tiled.restype = i64
            L.oracle_run_ghost_merge.argtypes = [i32, P, f64, f64, f64, f64, i32, u64,
                                                 f64, P, P, i64, i32, i64, P, P, P, P, P]
            L.oracle_run_ghost_merge.restype = i64
            _LIB = L
    return _LIB


def _p(a: np.ndarray) -> ctypes.c_void_p:
    assert a.flags["C_CONTIGUOUS"]
    return ctypes.c_void_p(a.ctypes.data)


def _dims(params) -> np.ndarray:
    L = list(params["L"]) + [1] * (3 - len(params["L"]))
    return np.asarray(L[:3], dtype=np.int32)


def n_cells(params) -> int:
    return int(np.prod([int(x) for x in params["L"][: params["dim"]]]))


# ---------------------------------------------------------------- primitives

def philox(counters: np.ndarray, seed: int) -> np.ndarray:
    """Philox4x32-10 of each row (c0, c1, c2, c3) under key (seed lo, seed hi)."""
    ctr = np.ascontiguousarray(counters, dtype=np.uint32).reshape(-1, 4)
    out = np.empty_like(ctr)
    lib().oracle_philox(_p(ctr), int(seed), _p(out), ctr.shape[0])
    return out


def neg_log_words(words: np.ndarray) -> np.ndarray:
    """E(u(w)) = -ln u for u = (2 (w >> 12) + 1) 2^-53, by the frozen recipe."""
    w = np.ascontiguousarray(words, dtype=np.uint64)
    out = np.empty(w.shape, dtype=np.float64)
    lib().oracle_neg_log_words(_p(w), _p(out), w.size)
    return out


def uniform_words(words: np.ndarray) -> np.ndarray:
    w = np.ascontiguousarray(words, dtype=np.uint64)
    out = np.empty(w.shape, dtype=np.float64)
    lib().oracle_uniform_words(_p(w), _p(out), w.size)
    return out


def ln2_split() -> tuple[float, float]:
    hi, lo = ctypes.c_double(), ctypes.c_double()
    lib().oracle_ln2_split(ctypes.byref(hi), ctypes.byref(lo))
    return hi.value, lo.value


def thresholds(dim: int, J: float, h: float, beta: float, rule: str,
               q: int = 1) -> np.ndarray:
    """Flip thresholds; q > 1 for the q-th degree neighbourhood's table."""
    out = np.zeros(130, dtype=np.uint64)
    if q > 1:
        k = lib().oracle_thresholds_range(int(dim), int(q), float(J), float(h),
                                          float(beta), RULES[rule], _p(out))
    else:
        k = lib().oracle_thresholds(int(dim), float(J), float(h), float(beta),
                                    RULES[rule], _p(out))
    if k < 0:
        raise ValueError("bad dimension or range")
    return out[:k].copy()


# ---------------------------------------------------------------- simulation

def init(params) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Initial (spins int8, first-arrival times f64, counts u32)."""
    N = n_cells(params)
    s = np.empty(N, dtype=np.int8)
    t = np.empty(N, dtype=np.float64)
    n = np.empty(N, dtype=np.uint32)
    dims = _dims(params)
    rc = lib().oracle_init(int(params["dim"]), _p(dims), float(params.get("rate", 1.0)),
                           INITS[params.get("init", "random")], int(params["seed"]),
                           _p(s), _p(t), _p(n))
    if rc != 0:
        raise ValueError("bad lattice parameters")
    return s, t, n


def run(params, T: float, s: np.ndarray, t: np.ndarray, n: np.ndarray):
    """Advance (s, t, n) in place to horizon T.  Returns (events, flips).
    params["range"] = q > 1 selects the q-th degree neighbourhood."""
    dims = _dims(params)
    q = int(params.get("range", 1))
    if q > 1:
        flips = ctypes.c_uint64(0)
        ev = lib().oracle_run_range(int(params["dim"]), _p(dims), q,
                                    float(params.get("J", 1.0)), float(params.get("h", 0.0)),
                                    float(params["beta"]), float(params.get("rate", 1.0)),
                                    RULES[params["rule"]], int(params["seed"]), float(T),
                                    _p(s), _p(t), _p(n), ctypes.byref(flips))
        if ev < 0:
            raise ValueError("bad lattice parameters")
        return int(ev), int(flips.value)
    flips = ctypes.c_uint64(0)
    ev = lib().oracle_run(int(params["dim"]), _p(dims), float(params.get("J", 1.0)),
                          float(params.get("h", 0.0)), float(params["beta"]),
                          float(params.get("rate", 1.0)), RULES[params["rule"]],
                          int(params["seed"]), float(T), _p(s), _p(t), _p(n),
                          ctypes.byref(flips))
    if ev < 0:
        raise ValueError("bad lattice parameters")
    return int(ev), int(flips.value)


def simulate(params, T: float):
    """init + run: the final (s, t, n) at horizon T and (events, flips)."""
    s, t, n = init(params)
    ev, fl = run(params, T, s, t, n)
    return s, t, n, ev, fl


def frames(params, T_start: float, T_end: float, dt: float, k_first: int, nframes: int,
           s: np.ndarray, t: np.ndarray, n: np.ndarray) -> dict:
    """Output frames (Fig. 3.7): advance (s, t, n) in place from T_start to T_end
    and return {k: spins at time k dt} for every k in [k_first, k_first + nframes)
    with k dt in (T_start, T_end].  The spins at time tau are the state after every
    arrival before tau, i.e. the state ``run`` leaves at horizon tau."""
    out = {}
    for k in range(k_first, k_first + nframes):
        tau = float(k) * dt
        if tau <= T_start or tau > T_end:
            continue
        run(params, tau, s, t, n)
        out[k] = s.copy()
    run(params, T_end, s, t, n)
    return out


def cell_clock(params, cells: np.ndarray, T: float):
    """Per-cell first arrival >= T and arrival count < T, from the cell's draws alone."""
    c = np.ascontiguousarray(cells, dtype=np.uint32)
    t = np.empty(c.shape, dtype=np.float64)
    n = np.empty(c.shape, dtype=np.uint32)
    lib().oracle_cell_clock(int(params["seed"]), float(params.get("rate", 1.0)), _p(c),
                            c.size, float(T), _p(t), _p(n))
    return t, n


def run_rounds(params, T: float, s, t, n, times_only: bool = False,
               max_record: int = 1 << 20):
    """Synchronous rounds (Fig. 3.2, index tie rule).  Returns
    (events, rounds, flips, enabled_per_round[:rounds])."""
    dims = _dims(params)
    rec = np.zeros(max_record, dtype=np.int64)
    rounds = ctypes.c_int64(0)
    flips = ctypes.c_uint64(0)
    ev = lib().oracle_run_rounds(int(params["dim"]), _p(dims), float(params.get("J", 1.0)),
                                 float(params.get("h", 0.0)), float(params["beta"]),
                                 float(params.get("rate", 1.0)), RULES[params["rule"]],
                                 int(params["seed"]), float(T), int(bool(times_only)),
                                 _p(s), _p(t), _p(n), _p(rec), max_record,
                                 ctypes.byref(rounds), ctypes.byref(flips))
    if ev < 0:
        raise ValueError("bad lattice parameters")
    r = int(rounds.value)
    return int(ev), r, int(flips.value), rec[: min(r, max_record)].copy()


def run_tiled(params, T: float, s, t, n, tile, max_rounds: int = 1 << 30,
              max_passes: int = 1 << 40):
    """Aggregated frozen-halo schedule (Fig. 3.4).  Returns
    (events, flips, passes, visits, rounds)."""
    dims = _dims(params)
    tl = np.asarray(list(tile) + [1] * (3 - len(tile)), dtype=np.int32)[:3]
    stats = np.zeros(3, dtype=np.int64)
    flips = ctypes.c_uint64(0)
    ev = lib().oracle_run_tiled(int(params["dim"]), _p(dims), float(params.get("J", 1.0)),
                                float(params.get("h", 0.0)), float(params["beta"]),
                                float(params.get("rate", 1.0)), RULES[params["rule"]],
                                int(params["seed"]), float(T), _p(tl), int(max_rounds),
                                int(max_passes), _p(s), _p(t), _p(n), _p(stats),
                                ctypes.byref(flips))
    if ev < 0:
        raise ValueError("bad lattice parameters")
    return int(ev), int(flips.value), int(stats[0]), int(stats[1]), int(stats[2])


def run_ghost_merge(params, T: float, s, t, n, tile, ghost, max_rounds: int = 1 << 30,
                    merge_ghosts: bool = True, max_launches: int = 1 << 40):
    """The GPU library's launch schedule (tiles + ghost zones against one snapshot,
    copies merged by most arrivals applied).  Returns (events, launches, rounds)."""
    dims = _dims(params)
    tl = np.asarray(list(tile) + [1] * (3 - len(tile)), dtype=np.int32)[:3]
    gh = np.asarray(list(ghost) + [0] * (3 - len(ghost)), dtype=np.int32)[:3]
    stats = np.zeros(2, dtype=np.int64)
    flips = ctypes.c_uint64(0)
    ev = lib().oracle_run_ghost_merge(int(params["dim"]), _p(dims),
                                      float(params.get("J", 1.0)), float(params.get("h", 0.0)),
                                      float(params["beta"]), float(params.get("rate", 1.0)),
                                      RULES[params["rule"]], int(params["seed"]), float(T),
                                      _p(tl), _p(gh), int(max_rounds), int(bool(merge_ghosts)),
                                      int(max_launches), _p(s), _p(t), _p(n), _p(stats),
                                      ctypes.byref(flips))
    if ev < 0:
        raise ValueError("bad lattice parameters")
    return int(ev), int(stats[0]), int(stats[1])
