"""MI355X-native central-moment lattice Boltzmann (CLB) for incompressible thermal flow.

The hot path -- one fused collide-and-stream pass per time step for the D2Q9 flow and D2Q5
temperature populations, with wall conditions and diagnostics -- is HIP code for gfx950 in
``csrc/``, built into ``libclb.so`` behind the C ABI declared in ``include/clb.h``.  ``clb`` is the
thin ctypes binding to it; ``workloads`` holds seeded synthetic problem descriptions.

Importing this package loads nothing; ``paper_1710_10569_amd.clb`` loads the library and fails
loudly if it has not been built.
"""
__all__ = ["clb", "workloads"]
