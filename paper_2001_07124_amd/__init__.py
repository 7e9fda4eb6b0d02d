"""Randomized HOSVD / R-STHOSVD on one MI355X (gfx950).

The compute path is the HIP library librhosvd.so (C ABI: include/rhosvd.h);
`paper_2001_07124_amd.api` is a thin ctypes binding over it that uses
PyTorch only for device memory and streams; `paper_2001_07124_amd.inputs`
draws seeded synthetic tensors.

Importing the package loads nothing; the first compute call loads the GPU
library and fails loudly if it is not built.
"""
