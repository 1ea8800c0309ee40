"""ctypes binding of libaca (include/aca.h): argument marshalling only.

Every step of the simulation runs in the library's HIP kernels; PyTorch only
provides device memory and the current stream.  ``load()`` raises when the
library is missing -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaca.so")

ACA_OK, ACA_EINVAL, ACA_ENOMEM, ACA_EDEVICE, ACA_ESTATE, ACA_ENOPROGRESS = 0, -1, -2, -3, -4, -5
RULES = {"glauber": 0, "metropolis": 1}
INITS = {"random": 0, "plus": 1, "minus": 2}

EXPORTED = ("aca_abi_version", "aca_last_error", "aca_thresholds", "aca_query",
            "aca_create", "aca_set_tuning", "aca_get_tuning", "aca_init", "aca_resume",
            "aca_advance", "aca_get_stats", "aca_read", "aca_destroy", "aca_philox",
            "aca_neg_log", "aca_batch_query", "aca_batch_create", "aca_batch_set_tuning",
            "aca_batch_get_tuning", "aca_batch_attach", "aca_batch_step", "aca_batch_poll",
            "aca_batch_advance", "aca_batch_members", "aca_batch_get_stats",
            "aca_batch_destroy", "aca_server_query", "aca_server_job_bytes",
            "aca_server_create", "aca_server_set_tuning", "aca_server_submit",
            "aca_server_step", "aca_server_job", "aca_server_read", "aca_server_release",
            "aca_server_load", "aca_server_get_stats", "aca_server_destroy", "aca_tune",
            "aca_batch_tune", "aca_batch_set_order", "aca_server_set_order",
            "aca_advance_frames", "aca_set_lag", "aca_get_thresholds", "aca_get_trace",
            "aca_advance_static", "aca_set_counting")
ORDER_WORK, ORDER_ARRIVAL = 0, 1
TUNE_MAX = 16
JOB_QUEUED, JOB_RUNNING, JOB_DONE, JOB_FAILED = 0, 1, 2, 3


class AcaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libaca error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("dim", ctypes.c_int32),
                ("L", ctypes.c_int32 * 3), ("J", ctypes.c_double), ("h", ctypes.c_double),
                ("beta", ctypes.c_double), ("rate", ctypes.c_double),
                ("rule", ctypes.c_int32), ("init", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("range", ctypes.c_int32),
                ("pad_", ctypes.c_int32)]


PARAMS_SIZE_V1 = 72     # aca_params without the range field (still accepted)


class Tuning(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("tile", ctypes.c_int32 * 3),
                ("ghost", ctypes.c_int32 * 3), ("max_sweeps", ctypes.c_int32),
                ("block", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("pad_", ctypes.c_uint32),
                ("launches", ctypes.c_uint64), ("visits", ctypes.c_uint64),
                ("sweeps", ctypes.c_uint64), ("events", ctypes.c_uint64),
                ("flips", ctypes.c_uint64), ("ghost_events", ctypes.c_uint64),
                ("cell_checks", ctypes.c_uint64), ("last_T", ctypes.c_double),
                ("device_ms", ctypes.c_double), ("kernel_ms", ctypes.c_double),
                ("region_bytes", ctypes.c_uint64), ("scan_live", ctypes.c_uint64),
                ("scan_enabled", ctypes.c_uint64), ("round_cells", ctypes.c_uint64)]


class LaunchRecord(ctypes.Structure):
    _fields_ = [("events", ctypes.c_uint64), ("ghost_events", ctypes.c_uint64),
                ("scan_live", ctypes.c_uint64), ("scan_enabled", ctypes.c_uint64),
                ("round_cells", ctypes.c_uint64), ("live_tiles", ctypes.c_uint64),
                ("kernel_ms", ctypes.c_double)]


TRACE_MAX = 65536


class BatchStats(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("pad_", ctypes.c_uint32),
                ("steps", ctypes.c_uint64), ("epochs", ctypes.c_uint64),
                ("visits", ctypes.c_uint64), ("sweeps", ctypes.c_uint64),
                ("events", ctypes.c_uint64), ("flips", ctypes.c_uint64),
                ("ghost_events", ctypes.c_uint64), ("cell_checks", ctypes.c_uint64),
                ("finished", ctypes.c_uint64), ("device_ms", ctypes.c_double),
                ("kernel_ms", ctypes.c_double), ("region_bytes", ctypes.c_uint64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("pad_", ctypes.c_uint32),
                ("submitted", ctypes.c_uint64), ("admitted", ctypes.c_uint64),
                ("finished", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("steps", ctypes.c_uint64), ("events", ctypes.c_uint64),
                ("arena_bytes", ctypes.c_uint64), ("arena_peak", ctypes.c_uint64),
                ("queued_peak", ctypes.c_uint64), ("device_ms", ctypes.c_double),
                ("kernel_ms", ctypes.c_double)]


_LIB = None


def load() -> ctypes.CDLL:
    """Load libaca.so (built in-tree by ``build.py``); raise if it is missing."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_cs_0502039_amd.build` (no fallback exists)")
    L = ctypes.CDLL(LIB_PATH)
    P, u64, i32, f64 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32, ctypes.c_double
    pp, pt, ps = ctypes.POINTER(Params), ctypes.POINTER(Tuning), ctypes.POINTER(Stats)
    L.aca_abi_version.restype = ctypes.c_uint32
    L.aca_abi_version.argtypes = []
    L.aca_last_error.restype = ctypes.c_char_p
    L.aca_last_error.argtypes = []
    sigs = {
        "aca_thresholds": [pp, P, i32, P],
        "aca_query": [pp, P, P],
        "aca_create": [pp, P, P, P, P, u64, P],
        "aca_set_tuning": [P, pt],
        "aca_get_tuning": [P, pt],
        "aca_init": [P, P],
        "aca_resume": [P, f64],
        "aca_advance": [P, f64, P],
        "aca_get_stats": [P, ps],
        "aca_read": [P, P, P, P, P],
        "aca_destroy": [P],
        "aca_philox": [P, u64, P, u64, P],
        "aca_neg_log": [P, P, u64, P],
        "aca_batch_query": [i32, P],
        "aca_batch_create": [i32, P, u64, P],
        "aca_batch_set_tuning": [P, i32, pt],
        "aca_batch_get_tuning": [P, i32, pt],
        "aca_batch_attach": [P, P, f64],
        "aca_batch_step": [P, f64, i32, P, P],
        "aca_batch_poll": [P, P, i32, P],
        "aca_batch_advance": [P, P, P, i32, P],
        "aca_batch_members": [P, P, i32, P],
        "aca_tune": [P, pt, i32, f64, P, P, P, P],
        "aca_batch_set_order": [P, i32],
        "aca_advance_frames": [P, f64, f64, P, ctypes.c_int64, ctypes.c_int64, P],
        "aca_set_lag": [P, f64],
        "aca_get_thresholds": [P, P, i32],
        "aca_get_trace": [P, ctypes.POINTER(LaunchRecord), i32, P],
        "aca_advance_static": [pp, P, P, P, i32, f64, f64, P],
        "aca_set_counting": [P, i32],
        "aca_server_set_order": [P, i32],
        "aca_batch_tune": [P, P, P, i32, i32, pt, i32, f64, P, P, P, P],
        "aca_batch_get_stats": [P, ctypes.POINTER(BatchStats)],
        "aca_batch_destroy": [P],
        "aca_server_query": [i32, P],
        "aca_server_job_bytes": [pp, P],
        "aca_server_create": [P, u64, P, u64, i32, P],
        "aca_server_set_tuning": [P, i32, pt],
        "aca_server_submit": [P, pp, f64, P],
        "aca_server_step": [P, f64, P, P, i32, P],
        "aca_server_job": [P, u64, P, ps],
        "aca_server_read": [P, u64, P, P, P, P],
        "aca_server_release": [P, u64],
        "aca_server_load": [P, P, P],
        "aca_server_get_stats": [P, ctypes.POINTER(ServerStats)],
        "aca_server_destroy": [P],
    }
    for name, args in sigs.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int32
    _LIB = L
    return L


def _check(code: int) -> None:
    if code != ACA_OK:
        raise AcaError(code, load().aca_last_error().decode(errors="replace"))


def make_params(p: dict) -> Params:
    L = list(p["L"]) + [1] * (3 - len(p["L"]))
    return Params(ctypes.sizeof(Params), int(p["dim"]), (ctypes.c_int32 * 3)(*L[:3]),
                  float(p.get("J", 1.0)), float(p.get("h", 0.0)), float(p["beta"]),
                  float(p.get("rate", 1.0)), RULES[p.get("rule", "glauber")],
                  INITS[p.get("init", "random")], int(p["seed"]) & (2**64 - 1),
                  int(p.get("range", 1)), 0)


def make_tuning(tile=(0, 0, 0), ghost=(-1, -1, -1), max_sweeps=0, block=0) -> Tuning:
    tile = list(tile) + [0] * (3 - len(tile))
    ghost = list(ghost) + [-1] * (3 - len(ghost))
    return Tuning(ctypes.sizeof(Tuning), (ctypes.c_int32 * 3)(*tile[:3]),
                  (ctypes.c_int32 * 3)(*ghost[:3]), int(max_sweeps), int(block))


def _tuning_array(candidates):
    """(Tuning array or None, count) for the autotuner entry points."""
    if not candidates:
        return None, 0
    arr = (Tuning * len(candidates))(*[make_tuning(**c) for c in candidates])
    return arr, len(candidates)


def abi_version() -> int:
    return int(load().aca_abi_version())


def thresholds(p: dict) -> np.ndarray:
    """The library's flip thresholds (host computation, no GPU needed)."""
    out = np.zeros(64, dtype=np.uint64)
    count = ctypes.c_int32(0)
    _check(load().aca_thresholds(ctypes.byref(make_params(p)), out.ctypes.data, 64,
                                 ctypes.byref(count)))
    return out[: count.value].copy()


def query(p: dict) -> tuple[int, int]:
    n = ctypes.c_uint64(0)
    sb = ctypes.c_uint64(0)
    _check(load().aca_query(ctypes.byref(make_params(p)), ctypes.byref(n), ctypes.byref(sb)))
    return int(n.value), int(sb.value)


def _stream_ptr(torch, stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class Lattice:
    """A lattice whose state lives in torch tensors on the GPU.

    ``spins`` (int8), ``times`` (float64) and ``counts`` (int32 storage holding
    uint32 values) are the caller-owned buffers of the C-ABI, in cell order
    x + L0 (y + L1 z).
    """

    def __init__(self, params: dict, device: str = "cuda", tuning: Optional[dict] = None,
                 stream=None):
        import torch
        self._torch = torch
        self.params = dict(params)
        self.lib = load()
        self.n, scratch = query(self.params)
        self.device = torch.device(device)
        self.stream = stream
        self.spins = torch.empty(self.n, dtype=torch.int8, device=self.device)
        self.times = torch.empty(self.n, dtype=torch.float64, device=self.device)
        self.counts = torch.empty(self.n, dtype=torch.int32, device=self.device)
        self.scratch = torch.empty(scratch, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        _check(self.lib.aca_create(ctypes.byref(make_params(self.params)),
                                   self.spins.data_ptr(), self.times.data_ptr(),
                                   self.counts.data_ptr(), self.scratch.data_ptr(),
                                   scratch, ctypes.byref(h)))
        self._h = h
        if tuning:
            self.set_tuning(**tuning)

    def _s(self) -> int:
        return _stream_ptr(self._torch, self.stream)

    def set_tuning(self, **kw) -> None:
        t = make_tuning(**kw) if kw else None
        _check(self.lib.aca_set_tuning(self._h, ctypes.byref(t) if t is not None else None))

    def tuning(self) -> dict:
        t = Tuning()
        _check(self.lib.aca_get_tuning(self._h, ctypes.byref(t)))
        return {"tile": list(t.tile), "ghost": list(t.ghost), "max_sweeps": t.max_sweeps,
                "block": t.block}

    def tune(self, dT: float, candidates=None) -> dict:
        """Advance by slices of dT, one candidate schedule per slice, and keep
        the fastest (results are the same whichever is chosen)."""
        cands, n = _tuning_array(candidates)
        best = ctypes.c_int32(0)
        count = ctypes.c_int32(0)
        rates = (ctypes.c_double * TUNE_MAX)()
        _check(self.lib.aca_tune(self._h, cands, n, float(dT), self._s(), ctypes.byref(best),
                                 rates, ctypes.byref(count)))
        return {"best": best.value, "rates_per_ms": list(rates[:count.value]),
                "tuning": self.tuning()}

    def init(self) -> "Lattice":
        _check(self.lib.aca_init(self._h, self._s()))
        return self

    def resume(self, T_done: float) -> None:
        _check(self.lib.aca_resume(self._h, float(T_done)))

    def advance(self, T: float) -> "Lattice":
        _check(self.lib.aca_advance(self._h, float(T), self._s()))
        return self

    def advance_frames(self, T: float, dt: float, frames, k_first: int) -> "Lattice":
        """Advance to T and fill frames[k] (an (nframes, N) int8 cuda tensor) with
        the spins at time (k_first + k) dt for the frame times in (last T, T]."""
        assert frames.dtype == self._torch.int8 and frames.is_contiguous()
        assert frames.numel() == 0 or frames.shape[-1] == self.n
        nframes = frames.shape[0] if frames.numel() else 0
        _check(self.lib.aca_advance_frames(self._h, float(T), float(dt),
                                           frames.data_ptr() if nframes else None,
                                           int(k_first), int(nframes), self._s()))
        return self

    def set_counting(self, on: bool = True) -> "Lattice":
        """Collect the Section 4 efficiency counters in later advances."""
        _check(self.lib.aca_set_counting(self._h, 1 if on else 0))
        return self

    def set_lag(self, lag: float) -> None:
        _check(self.lib.aca_set_lag(self._h, float(lag)))

    def stats(self) -> dict:
        st = Stats()
        st.struct_size = ctypes.sizeof(Stats)
        _check(self.lib.aca_get_stats(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in Stats._fields_ if k not in ("struct_size", "pad_")}

    def thresholds(self) -> np.ndarray:
        """The flip thresholds this lattice applies."""
        out = np.zeros(64, dtype=np.uint64)
        _check(self.lib.aca_get_thresholds(self._h, out.ctypes.data, 64))
        return out[: thresholds(self.params).size].copy()

    def trace(self) -> list[dict]:
        """Per-launch records of the last advance (efficiency per launch)."""
        count = ctypes.c_int32(0)
        _check(self.lib.aca_get_trace(self._h, None, 0, ctypes.byref(count)))
        buf = (LaunchRecord * max(1, count.value))()
        _check(self.lib.aca_get_trace(self._h, buf, count.value, ctypes.byref(count)))
        return [{k: getattr(buf[i], k) for k, _ in LaunchRecord._fields_}
                for i in range(count.value)]

    def read(self) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
        """Synchronous copy of (spins int8, times float64, counts uint32) to the host."""
        s = np.empty(self.n, dtype=np.int8)
        t = np.empty(self.n, dtype=np.float64)
        c = np.empty(self.n, dtype=np.uint32)
        _check(self.lib.aca_read(self._h, s.ctypes.data, t.ctypes.data, c.ctypes.data,
                                 self._s()))
        return s, t, c

    def close(self) -> None:
        if getattr(self, "_h", None):
            self.lib.aca_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many lattices advanced together by the persistent batch kernel.

    Attached ``Lattice`` objects are kept alive by the batch until they are
    returned by ``poll`` (or ``advance`` returns), since the device works on
    their buffers meanwhile.
    """

    def __init__(self, capacity: int, device: str = "cuda", stream=None):
        import torch
        self._torch = torch
        self.lib = load()
        self.capacity = int(capacity)
        nbytes = ctypes.c_uint64(0)
        _check(self.lib.aca_batch_query(self.capacity, ctypes.byref(nbytes)))
        self.work = torch.empty(int(nbytes.value), dtype=torch.uint8, device=device)
        self.stream = stream
        h = ctypes.c_void_p()
        _check(self.lib.aca_batch_create(self.capacity, self.work.data_ptr(),
                                         int(nbytes.value), ctypes.byref(h)))
        self._h = h
        self._members: dict[int, "Lattice"] = {}

    def _s(self) -> int:
        return _stream_ptr(self._torch, self.stream)

    def set_tuning(self, dim: int, **kw) -> None:
        t = make_tuning(**kw) if kw else None
        _check(self.lib.aca_batch_set_tuning(self._h, int(dim),
                                             ctypes.byref(t) if t is not None else None))

    def tuning(self, dim: int) -> dict:
        t = Tuning()
        _check(self.lib.aca_batch_get_tuning(self._h, int(dim), ctypes.byref(t)))
        return {"tile": list(t.tile), "ghost": list(t.ghost), "max_sweeps": t.max_sweeps,
                "block": t.block}

    def tune(self, lattices, T, dim: int, candidates=None, frac: float = 0.02) -> dict:
        """Advance the lattices (towards horizons T) slice by slice, one
        candidate schedule for dimension `dim` per slice, and keep the fastest."""
        lats = list(lattices)
        Ts = np.asarray(T, dtype=np.float64)
        handles = (ctypes.c_void_p * len(lats))(*[l._h.value for l in lats])
        cands, n = _tuning_array(candidates)
        best = ctypes.c_int32(0)
        count = ctypes.c_int32(0)
        rates = (ctypes.c_double * TUNE_MAX)()
        for l in lats:
            self._members[l._h.value] = l
        try:
            _check(self.lib.aca_batch_tune(self._h, handles, Ts.ctypes.data, len(lats),
                                           int(dim), cands, n, float(frac), self._s(),
                                           ctypes.byref(best), rates, ctypes.byref(count)))
        finally:
            for l in lats:
                self._members.pop(l._h.value, None)
        return {"best": best.value, "rates_per_ms": list(rates[:count.value]),
                "tuning": self.tuning(dim)}

    def set_order(self, order: int) -> None:
        _check(self.lib.aca_batch_set_order(self._h, int(order)))

    def attach(self, lat: "Lattice", T: float) -> None:
        _check(self.lib.aca_batch_attach(self._h, lat._h, float(T)))
        self._members[lat._h.value] = lat

    def step(self, budget_ms: float = 0.0, max_epochs: int = 0) -> int:
        """One persistent launch; returns the number of members still attached."""
        left = ctypes.c_int32(0)
        code = self.lib.aca_batch_step(self._h, float(budget_ms), int(max_epochs), self._s(),
                                       ctypes.byref(left))
        if code != ACA_OK:
            msg = self.lib.aca_last_error().decode(errors="replace")
            self._forget_detached()
            raise AcaError(code, msg)
        return int(left.value)

    def _forget_detached(self) -> None:
        buf = (ctypes.c_void_p * max(1, self.capacity))()
        n = ctypes.c_int32(0)
        _check(self.lib.aca_batch_members(self._h, buf, self.capacity, ctypes.byref(n)))
        keep = {buf[i] for i in range(n.value)}
        for key in list(self._members):
            if key not in keep:
                del self._members[key]

    def poll(self) -> list:
        """Lattices that reached their horizon since the last poll."""
        out = []
        buf = (ctypes.c_void_p * 64)()
        n = ctypes.c_int32(0)
        while True:
            _check(self.lib.aca_batch_poll(self._h, buf, 64, ctypes.byref(n)))
            for i in range(n.value):
                out.append(self._members.pop(buf[i]))
            if n.value < 64:
                return out

    def advance(self, lattices, T) -> None:
        """Advance lattices[i] to T[i] in one batch (which must be empty)."""
        lats = list(lattices)
        Ts = np.asarray(T, dtype=np.float64)
        if Ts.shape != (len(lats),):
            raise ValueError("one horizon per lattice")
        handles = (ctypes.c_void_p * max(1, len(lats)))(*[l._h.value for l in lats])
        for l in lats:
            self._members[l._h.value] = l
        try:
            _check(self.lib.aca_batch_advance(self._h, handles, Ts.ctypes.data, len(lats),
                                              self._s()))
        finally:
            for l in lats:
                self._members.pop(l._h.value, None)

    def stats(self) -> dict:
        st = BatchStats()
        st.struct_size = ctypes.sizeof(BatchStats)
        _check(self.lib.aca_batch_get_stats(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in BatchStats._fields_
                if k not in ("struct_size", "pad_")}

    def close(self) -> None:
        if getattr(self, "_h", None):
            _check(self.lib.aca_batch_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def job_bytes(p: dict) -> int:
    """Arena bytes a served job with parameters p occupies."""
    out = ctypes.c_uint64(0)
    _check(load().aca_server_job_bytes(ctypes.byref(make_params(p)), ctypes.byref(out)))
    return int(out.value)


class Server:
    """Continuous batching of simulation jobs over a device arena (HBM budget)."""

    def __init__(self, arena_bytes: int, max_jobs: int = 256, device: str = "cuda",
                 stream=None):
        import torch
        self._torch = torch
        self.lib = load()
        self.max_jobs = int(max_jobs)
        wb = ctypes.c_uint64(0)
        _check(self.lib.aca_server_query(self.max_jobs, ctypes.byref(wb)))
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=device)
        self.work = torch.empty(int(wb.value), dtype=torch.uint8, device=device)
        self.stream = stream
        h = ctypes.c_void_p()
        _check(self.lib.aca_server_create(self.arena.data_ptr(), int(arena_bytes),
                                          self.work.data_ptr(), int(wb.value), self.max_jobs,
                                          ctypes.byref(h)))
        self._h = h
        self._done = (ctypes.c_uint64 * self.max_jobs)()
        self._n = {}

    def _s(self) -> int:
        return _stream_ptr(self._torch, self.stream)

    def set_tuning(self, dim: int, **kw) -> None:
        t = make_tuning(**kw) if kw else None
        _check(self.lib.aca_server_set_tuning(self._h, int(dim),
                                              ctypes.byref(t) if t is not None else None))

    def set_order(self, order: int) -> None:
        _check(self.lib.aca_server_set_order(self._h, int(order)))

    def submit(self, params: dict, T: Optional[float] = None) -> int:
        job = ctypes.c_uint64(0)
        _check(self.lib.aca_server_submit(self._h, ctypes.byref(make_params(params)),
                                          float(params["T"] if T is None else T),
                                          ctypes.byref(job)))
        self._n[job.value] = query(params)[0]
        return int(job.value)

    def step(self, budget_ms: float = 0.0) -> list:
        """Admit what fits, run one batch step; returns ids of jobs that finished."""
        n = ctypes.c_int32(0)
        _check(self.lib.aca_server_step(self._h, float(budget_ms), self._s(), self._done,
                                        self.max_jobs, ctypes.byref(n)))
        return [int(self._done[i]) for i in range(min(n.value, self.max_jobs))]

    def job(self, job: int) -> tuple[int, dict]:
        state = ctypes.c_int32(0)
        st = Stats()
        st.struct_size = ctypes.sizeof(Stats)
        _check(self.lib.aca_server_job(self._h, int(job), ctypes.byref(state),
                                       ctypes.byref(st)))
        return int(state.value), {k: getattr(st, k) for k, _ in Stats._fields_
                                  if k not in ("struct_size", "pad_")}

    def read(self, job: int) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
        n = self._n[job]
        s = np.empty(n, dtype=np.int8)
        t = np.empty(n, dtype=np.float64)
        c = np.empty(n, dtype=np.uint32)
        _check(self.lib.aca_server_read(self._h, int(job), s.ctypes.data, t.ctypes.data,
                                        c.ctypes.data, self._s()))
        return s, t, c

    def release(self, job: int) -> None:
        _check(self.lib.aca_server_release(self._h, int(job)))
        self._n.pop(job, None)

    def load(self) -> tuple[int, int]:
        q = ctypes.c_int32(0)
        r = ctypes.c_int32(0)
        _check(self.lib.aca_server_load(self._h, ctypes.byref(q), ctypes.byref(r)))
        return int(q.value), int(r.value)

    def stats(self) -> dict:
        st = ServerStats()
        st.struct_size = ctypes.sizeof(ServerStats)
        _check(self.lib.aca_server_get_stats(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in ServerStats._fields_
                if k not in ("struct_size", "pad_")}

    def close(self) -> None:
        if getattr(self, "_h", None):
            _check(self.lib.aca_server_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def philox(counters, seed: int, stream=None):
    """Philox4x32-10 on the GPU: counters is an (n, 4) int32/uint32 tensor on cuda."""
    import torch
    ctr = counters.contiguous()
    out = torch.empty_like(ctr)
    _check(load().aca_philox(ctr.data_ptr(), int(seed) & (2**64 - 1), out.data_ptr(),
                             ctr.shape[0], _stream_ptr(torch, stream)))
    return out


def neg_log(words, stream=None):
    """-ln u(w) on the GPU for a uint64 (int64 storage) tensor on cuda."""
    import torch
    w = words.contiguous()
    out = torch.empty(w.shape, dtype=torch.float64, device=w.device)
    _check(load().aca_neg_log(w.data_ptr(), out.data_ptr(), w.numel(),
                              _stream_ptr(torch, stream)))
    return out


def advance_static(params: dict, spins, times, counts, T: float, T_done: float = 0.0,
                   draw_initial: bool = False, stream=None) -> None:
    """Allocation-free advance of caller tensors (int8, float64, int32 storage
    holding uint32; N elements each on cuda) from T_done to T, drawing the
    initial state first when draw_initial is set."""
    import torch
    for x, dt in ((spins, torch.int8), (times, torch.float64), (counts, torch.int32)):
        assert x.dtype == dt and x.is_contiguous() and x.is_cuda
    _check(load().aca_advance_static(ctypes.byref(make_params(params)), spins.data_ptr(),
                                     times.data_ptr(), counts.data_ptr(),
                                     1 if draw_initial else 0, float(T_done), float(T),
                                     _stream_ptr(torch, stream)))


def simulate(params: dict, T: Optional[float] = None, tuning: Optional[dict] = None):
    """init + advance to T (default params["T"]); returns host (s, t, n) and stats."""
    lat = Lattice(params, tuning=tuning)
    lat.init().advance(params["T"] if T is None else T)
    s, t, n = lat.read()
    st = lat.stats()
    lat.close()
    return s, t, n, st
