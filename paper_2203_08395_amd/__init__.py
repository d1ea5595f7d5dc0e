"""MI355X (gfx950) levelized static timing analysis.

``sta``  -- binding of libsta.so (the C ABI in include/sta.h): graph build, RC delay
           calculation, forward propagation, required times and slack, all on the GPU.
``gen``  -- seeded synthetic designs, libraries and per-view inputs.
``build``-- compiles libsta.so with hipcc for gfx950.
"""
__all__ = ["sta", "gen", "build"]
