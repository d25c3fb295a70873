"""MI355X (gfx950) implementation of the NUMARCK compression hot path
("Parallel Implementation of Lossy Data Compression for Temporal Data Sets",
Yuan et al., arXiv 1703.02438).

The compute path is the HIP library ``libnumarck.so`` (C ABI in
``include/numarck.h``); :mod:`paper_1703_02438_amd.numarck` is its thin
Python binding.  Importing that module fails if the library is not built.
"""
