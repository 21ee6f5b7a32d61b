"""Block-sparse U(1)xU(1) two-site DMRG hot path on AMD MI355X (gfx950).

The compute lives in libbsdmrg.so (C ABI in include/bsdmrg.h); the binding
module `paper_2412_04676_amd.bsdmrg` loads it.  Importing this package does
not load the library, so `build` can run without it.
"""
