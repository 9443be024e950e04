"""FP64 CPU oracle for the Fourier-subsampled pulse-echo operator and its solvers.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this package:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It shares no code, tables or constants with the HIP
library; the two meet only through the seeded inputs of the workload module
(which holds none of the method's arithmetic) and through numbers written
out by the paper.

The oracle is deliberately plain and slow: it writes out the definition of
each quantity in float64 / complex128 with numpy, with no blocking, no FFT
tricks, no integer-phase arithmetic and no Toeplitz reuse.

Modules
-------
geometry   pulse spectrum, band, grids, round-trip delay, window start
select     SplitMix64 bin selection (random draw inside the pulse band)
operator   the operator A (dense and per-position blocks), A x and A^H y
timedomain periodised time-domain A-scans (for the DFT cross-check)
solver     soft threshold, ISTA / FISTA, lambda rule, Lipschitz constant
learned    unrolled shrinkage network: forward pass and finite differences

Readings of passages where the paper is silent or garbled are listed in the
docstring of the function that takes them.
"""
