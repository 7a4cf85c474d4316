"""AES (FIPS-197) ECB/CTR on MI355X: hand-written gfx950 kernels behind the
C ABI of include/aesgpu.h.

The binding is the submodule ``paper_1403_7295_amd.aesgpu``; it loads the
library when imported (and raises if it is not built).
"""
