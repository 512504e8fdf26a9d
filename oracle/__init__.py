"""Plain FP64 CPU oracle for convolutional gridding.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import, call, link or execute anything in this
directory.  The GPU library never uses it, shares no code with it, and must
fail loudly rather than fall back to it.

Contents
--------
``gridding.py``   NumPy FP64: kernel tables (Kaiser-Bessel, separable and 2-D
                  W kernels), the uvw -> pixel/oversample/plane conversion with
                  its drop rule, and gridding written as its plain definition.
``grid_ref.c``    The same definition in C (FP64, OpenMP, threads own row
                  stripes, so results are deterministic), for full-size inputs,
                  sampled-row checks and CPU timing.  ``cgrid.py`` loads it.
"""
