"""MI355X-native conservative simulation of Poisson-asynchronous cellular arrays.

The continuous-time Ising model (Glauber or Metropolis rule) simulated by the
conservative parallel method of Lubachevsky, "Efficient Parallel Simulations of
Asynchronous Cellular Arrays": every cell keeps its own clock and applies its
next arrival only once no neighbour's clock lies behind it.  The update sweep is
hand-written HIP for gfx950 behind the C-ABI library ``libaca.so``; this package
is its thin ctypes binding (``paper_cs_0502039_amd.aca``) plus the seeded
workload generators (``paper_cs_0502039_amd.workloads``).

Importing the package loads nothing native; ``aca.load()`` does, and fails
loudly when the library is missing.
"""
