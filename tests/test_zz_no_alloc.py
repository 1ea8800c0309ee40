"""The allocation-free advance (aca_advance_static) against aca_advance.

Both run the same kernels; the allocation-free entry point keeps its working
snapshots, tile flags and counters in the library's fixed device array rather
than a caller scratch buffer.  Its results must equal those of
aca_create + aca_init/aca_resume + aca_advance bit for bit (the trajectory is
unique, argument after Fig. 3.1), on consecutive calls whose lattices shrink, so
that a call that left more of the array written than the next one reads would
show up.
"""
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


def state_tensors(torch, n):
    return (torch.empty(n, dtype=torch.int8, device="cuda"),
            torch.empty(n, dtype=torch.float64, device="cuda"),
            torch.empty(n, dtype=torch.int32, device="cuda"))


def host(tensors):
    s, t, c = tensors
    return (s.cpu().numpy(), t.cpu().numpy(), c.cpu().numpy().view(np.uint32))


def assert_same(a, b, label):
    for x, y, what in zip(a, b, ("spins", "times", "counts")):
        bad = np.flatnonzero(x.view(np.uint8 if x.dtype == np.int8 else x.dtype)
                             != y.view(np.uint8 if y.dtype == np.int8 else y.dtype))
        assert bad.size == 0, f"{label}: {bad.size} {what} differ, first cells {bad[:5]}"


def reference(params, T):
    s, t, n, _ = aca.simulate(params, T)
    return s, t, n


# larger lattice first, then smaller ones: later calls must not read what
# earlier ones left in the shared array
CASES = [
    ("2d_300x200", workloads.lattice(2, (300, 200), 0.4, "glauber", seed=7), 6.0),
    ("3d_20x18x16", workloads.lattice(3, (20, 18, 16), 0.22, "metropolis", h=0.1, seed=8,
                                      init="plus"), 4.0),
    ("2d_37x29", workloads.lattice(2, (37, 29), 0.44, "metropolis", seed=9), 5.0),
]


def test_static_advance_equals_handle_advance(torch):
    for label, params, T in CASES:
        say(f"no-alloc: {label} T={T}")
        n = aca.query(params)[0]
        x = state_tensors(torch, n)
        aca.advance_static(params, *x, T=T, draw_initial=True)
        got = host(x)
        assert_same(got, reference(params, T), label)
        if n <= 6000:
            os_, ot, on, _, _ = oracle.simulate(params, T)
            assert_same(got, (os_, ot, on), label + " vs oracle")


def test_static_advance_resumes_in_chunks(torch):
    """Two calls in a row on one state, the second smaller in span: from the
    initial state to T/2, then from T/2 to T (a restored state)."""
    for label, params, T in CASES[::-1]:
        say(f"no-alloc chunks: {label} T={T}")
        n = aca.query(params)[0]
        x = state_tensors(torch, n)
        aca.advance_static(params, *x, T=T / 2, draw_initial=True)
        aca.advance_static(params, *x, T=T, T_done=T / 2)
        assert_same(host(x), reference(params, T), label)


def test_static_advance_rejects_oversized_lattice(torch):
    params = workloads.lattice(2, (2048, 2048), 0.4, seed=1)
    x = state_tensors(torch, 16)
    with pytest.raises(aca.AcaError) as e:
        aca.advance_static(params, *x, T=1.0, draw_initial=True)
    assert e.value.code == aca.ACA_EINVAL and "static scratch" in str(e.value)
