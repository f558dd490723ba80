"""MI355X (gfx950) EIS-inversion grid search for PRNU source identification of
stabilised videos (arXiv 2207.14507).

The compute path is the HIP library ``libprnu.so`` behind the C ABI in
``include/prnu.h``; ``paper_2207_14507_amd.prnu`` is its ctypes binding (importing it
fails when the library has not been built), ``paper_2207_14507_amd.build`` builds it,
and ``paper_2207_14507_amd.synth`` draws the seeded synthetic workloads.
"""
__all__ = ["build", "prnu", "synth"]
