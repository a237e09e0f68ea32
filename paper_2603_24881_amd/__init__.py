"""MI355X-native multigrid Gaussian-plane-wave collocation / integration.

``_lib`` is the ctypes binding of libgpw.so (include/gpw.h); ``gpw.GPW`` binds a
plan to a system; ``synth`` draws the seeded synthetic workloads.
"""
