"""MI355X-native Fourier-subsampled pulse-echo reconstruction (arXiv 2012.04534).

The compute path is the HIP library ``libufss.so`` (sources in ``csrc/``,
C ABI in ``include/ufss.h``); ``ufss`` is its thin ctypes binding and
``workloads`` holds the synthetic inputs.  Importing the package does not load
the library; the first call through ``ufss`` does, and fails loudly if it is
missing.
"""
