"""MI355X-native simulator for Spiking Neural P systems with delays.

The hot path is a C-ABI HIP library (``csrc/``, declared in ``include/snp.h``);
``binding`` is its thin ctypes binding and ``workloads`` draws seeded synthetic
systems.  Importing this package does not load the library; importing
``paper_2408_04343_amd.binding`` does, and fails loudly if it is not built.
"""
